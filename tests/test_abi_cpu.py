"""CPU-side checks of the C ABI library: it loads and exports every symbol
include/qtt.h declares (no compute call is made without a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtt.h")
LIB = os.path.join(ROOT, "paper_1511_06029_amd", "libqtt.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qtt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("qtt_matrix_load", "qtt_apply", "qtt_solve", "qtt_apply_batched"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqtt.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(qtt_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqtt.so not built")
def test_binding_loads_and_matches_header():
    import torch  # noqa: F401  (shares its HIP runtime with the library)
    from paper_1511_06029_amd import qtt
    assert sorted(qtt.EXPORTED) == declared()
    assert qtt.lib().qtt_status_string(5) == b"not converged"
    # argument errors are reported before any device work
    import ctypes
    h = ctypes.c_void_p()
    r = (ctypes.c_int64 * 2)(2, 1)
    m = (ctypes.c_int64 * 1)(8)
    st = qtt.lib().qtt_matrix_load(1, r, m, m, (ctypes.c_void_p * 1)(None), 1, ctypes.byref(h))
    assert st == 2 and b"boundary" in qtt.lib().qtt_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqtt.so not built")
def test_solve_schedule_argument_errors():
    """qtt_solve_schedule rejects null handles before any device work (the
    pass-count check needs valid handles and runs on the GPU tests)."""
    import torch  # noqa: F401
    from paper_1511_06029_amd import qtt
    L = qtt.lib()
    st = L.qtt_solve_schedule(None, None, 1, None, 1, None, 1, None, 1, 1e-8, 4, None, 0, None, None)
    assert st == 1 and b"null handle" in L.qtt_last_error()    # QTT_ERR_INVALID_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqtt.so not built")
def test_schedule_struct_layout(tmp_path):
    """The binding's qtt_schedule_t has the C layout the header gives it
    (size and field offsets as compiled by gcc)."""
    import ctypes
    import torch  # noqa: F401
    from paper_1511_06029_amd import qtt
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "qtt.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu %zu %zu %zu", sizeof(qtt_schedule_t), '
                   'offsetof(qtt_schedule_t, inv_first), offsetof(qtt_schedule_t, first_compute), '
                   'offsetof(qtt_schedule_t, first_passes), offsetof(qtt_schedule_t, A_lo), '
                   'offsetof(qtt_schedule_t, lo_compute), offsetof(qtt_schedule_t, lo_below)); return 0; }\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    c = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    S = qtt._Schedule
    py = [ctypes.sizeof(S)] + [getattr(S, f).offset for f, _ in S._fields_]
    assert c == py, (c, py)
