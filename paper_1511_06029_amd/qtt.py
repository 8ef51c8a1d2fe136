"""Python binding of libqtt (ctypes).  Argument marshalling only: every step of
the apply and of the solve runs in the HIP library.  PyTorch supplies device
memory and streams.

Vectors are FP64 CUDA tensors.  A block of K vectors of length N is an
(N, K) tensor in column-major layout (``stride(0) == 1``, column stride
``stride(1) >= N``), e.g. ``empty_block(N, K)``; a single vector may be 1-D.

Importing this module loads ``libqtt.so`` from the package directory and
raises if it has not been built (``python -m paper_1511_06029_amd.build_lib``).
"""
from __future__ import annotations

import ctypes
import functools
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqtt.so")

QTT_FP64, QTT_FP32, QTT_BF16 = 1, 2, 4
DTYPES = {"fp64": QTT_FP64, "fp32": QTT_FP32, "bf16": QTT_BF16}

# configuration ids under which launches of the fused core pairs are timed:
# FP64 90.., FP32 100.. (+ 4 first core + 2 padded rank-32 kernel + rows of
# the second core above 192)
PAIR_SHAPES = list(range(90, 98)) + list(range(100, 108))
# FP32 interior cores with products formed from split BF16 operands (pinned only)
F32_SPLIT = 38

QTT_OK = 0
QTT_ERR_NOT_CONVERGED = 5
QTT_ERR_NONFINITE = 6


class QttError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"libqtt error {status}: {message}")
        self.status = status


class _SolveCol(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("rel_residual", ctypes.c_double)]


class _Schedule(ctypes.Structure):
    """qtt_schedule_t."""
    _fields_ = [("inv_first", ctypes.c_void_p), ("first_compute", ctypes.c_int32), ("first_passes", ctypes.c_int32),
                ("A_lo", ctypes.c_void_p), ("lo_compute", ctypes.c_int32), ("lo_below", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1511_06029_amd.build_lib` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32, SZ, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                               ctypes.c_uint32, ctypes.c_size_t, ctypes.c_double)
    PP = ctypes.POINTER(ctypes.c_void_p)
    PI64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "qtt_matrix_load": [I32, PI64, PI64, PI64, PP, U32, PP],
        "qtt_matrix_free": [P],
        "qtt_matrix_set_diagonals": [P, D, P, P],
        "qtt_matvec_compressed": [P, I64, PI64, PP, PP, P],
        "qtt_matrix_info": [P, ctypes.POINTER(I32), PI64, PI64, PI64, ctypes.POINTER(U32)],
        "qtt_workspace_bytes": [P, I32, I64, ctypes.POINTER(SZ)],
        "qtt_apply": [P, I32, I64, P, I64, P, I64, P, SZ, P],
        "qtt_apply_batched": [P, I32, I32, PI64, PP, PI64, PP, PI64, P, SZ, P],
        "qtt_apply_noalloc": [P, I32, I64, P, I64, P, I64, P],
        "qtt_autotune": [P, I32, I64, P, I64, P, I64, P, SZ, P],
        "qtt_solve_workspace_bytes": [P, P, I32, I64, ctypes.POINTER(SZ)],
        "qtt_solve": [P, P, I32, I64, P, I64, P, I64, D, I32, P, SZ, P, ctypes.POINTER(_SolveCol)],
        "qtt_solve_schedule": [P, P, I32, ctypes.POINTER(_Schedule), I64, P, I64, P, I64, D, I32, P, SZ, P,
                               ctypes.POINTER(_SolveCol)],
        "qtt_solve_schedule_workspace_bytes": [P, P, I32, ctypes.POINTER(_Schedule), I64, ctypes.POINTER(SZ)],
        "qtt_fgmres_workspace_bytes": [P, P, I32, I64, I32, ctypes.POINTER(SZ)],
        "qtt_solve_fgmres": [P, P, I32, I64, P, I64, P, I64, D, I32, P, SZ, P, ctypes.POINTER(_SolveCol)],
        "qtt_solve_fgmres_product": [P, P, P, I32, I64, P, I64, P, I64, D, I32, P, SZ, P,
                                     ctypes.POINTER(_SolveCol)],
        "qtt_fgmres_schedule_workspace_bytes": [P, P, I32, ctypes.POINTER(_Schedule), I64, I32, ctypes.POINTER(SZ)],
        "qtt_solve_fgmres_schedule": [P, P, I32, ctypes.POINTER(_Schedule), I64, P, I64, P, I64, D, I32, P, SZ, P,
                                      ctypes.POINTER(_SolveCol)],
        "qtt_set_shape": [P, I32, I32, I32],
        "qtt_list_shapes": [I32, ctypes.POINTER(I32), I32, ctypes.POINTER(I32)],
        "qtt_tt_round": [I32, PI64, PI64, PP, D, I32, ctypes.c_uint64, PP, PI64, P],
        "qtt_tt_compress": [I32, PI64, P, D, I32, ctypes.c_uint64, PP, PI64, P],
        "qtt_matrix_cores": [P, PP],
        "qtt_matrix_shape": [P, PI64, PI64, PI64],
        "qtt_invert_newton_schulz": [P, P, D, I32, I32, D, D, ctypes.c_uint64, U32, PP, ctypes.POINTER(D),
                                     ctypes.POINTER(I32), P],
        "qtt_timing_enable": [I32],
        "qtt_timing_reset": [],
        "qtt_timing_read": [I32, I32, PI64, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)],
        "qtt_timing_read_shape": [I32, I32, PI64, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.qtt_status_string.argtypes = [ctypes.c_int]
    lib.qtt_status_string.restype = ctypes.c_char_p
    lib.qtt_last_error.argtypes = []
    lib.qtt_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()
# Names the C ABI exports (include/qtt.h); the tests check each is present.
EXPORTED = ["qtt_matrix_load", "qtt_matrix_free", "qtt_matrix_set_diagonals", "qtt_matrix_info", "qtt_workspace_bytes",
            "qtt_apply", "qtt_apply_batched", "qtt_apply_noalloc", "qtt_autotune", "qtt_solve_workspace_bytes",
            "qtt_matvec_compressed", "qtt_solve", "qtt_solve_schedule", "qtt_solve_schedule_workspace_bytes", "qtt_fgmres_workspace_bytes", "qtt_solve_fgmres", "qtt_solve_fgmres_product", "qtt_fgmres_schedule_workspace_bytes", "qtt_solve_fgmres_schedule", "qtt_status_string", "qtt_last_error", "qtt_set_shape", "qtt_list_shapes",
            "qtt_tt_round", "qtt_tt_compress", "qtt_matrix_cores", "qtt_matrix_shape", "qtt_invert_newton_schulz",
            "qtt_timing_enable",
            "qtt_timing_reset", "qtt_timing_read", "qtt_timing_read_shape"]


def lib():
    return _lib


def _check(status, allow=()):
    if status != QTT_OK and status not in allow:
        raise QttError(status, _lib.qtt_last_error().decode())
    return status


def _dtype(compute):
    if isinstance(compute, str):
        return DTYPES[compute]
    return int(compute)


def _on_stream(fn):
    """Run a wrapper with its stream argument resolved and made torch's
    current stream, so that the temporaries it allocates (workspaces, and
    outputs it creates) belong to the stream the library enqueues on: the
    caching allocator then reuses their memory only behind that work."""
    @functools.wraps(fn)
    def wrapper(*args, stream=None, **kw):
        s = torch.cuda.current_stream() if stream is None else stream
        with torch.cuda.stream(s):
            return fn(*args, stream=s, **kw)
    return wrapper


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _col_major(T, name):
    """(ptr, rows, ncols, ld) of an FP64 CUDA tensor in column-major layout."""
    if not isinstance(T, torch.Tensor) or not T.is_cuda or T.dtype != torch.float64:
        raise TypeError(f"{name} must be an FP64 CUDA tensor")
    if T.dim() == 1:
        if T.stride(0) != 1:
            raise ValueError(f"{name} must be contiguous")
        return T.data_ptr(), T.shape[0], 1, T.shape[0]
    if T.dim() != 2 or (T.stride(0) != 1 and T.shape[0] > 1):
        raise ValueError(f"{name} must be an (N, K) column-major tensor (stride(0) == 1)")
    ld = T.stride(1) if T.shape[1] > 1 else T.shape[0]
    return T.data_ptr(), T.shape[0], T.shape[1], max(ld, T.shape[0])


def empty_block(N, K, device="cuda"):
    """Uninitialised (N, K) FP64 column-major tensor."""
    return torch.empty((K, N), dtype=torch.float64, device=device).t()


def to_block(X_np, device="cuda"):
    """Column-major device copy of a host (N,) or (N, K) array."""
    X_np = np.asarray(X_np, dtype=np.float64)
    if X_np.ndim == 1:
        return torch.from_numpy(X_np.copy()).to(device)
    return torch.from_numpy(np.ascontiguousarray(X_np.T)).to(device).t()


class QttMatrix:
    """A QTT matrix resident on the current device (handle from qtt_matrix_load)."""

    def __init__(self, handle, cores_shape):
        self._h = handle
        self.ranks, self.m, self.n = cores_shape
        self.d = len(self.m)
        self.rows = int(np.prod(self.m))
        self.cols = int(np.prod(self.n))

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("matrix was freed")
        return self._h

    def free(self):
        if self._h is not None:
            _check(_lib.qtt_matrix_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @classmethod
    def _from_handle(cls, h):
        """Wrap a handle the library created (shapes read back from it)."""
        hv = ctypes.c_void_p(h)
        d = ctypes.c_int32()
        _check(_lib.qtt_matrix_info(hv, ctypes.byref(d), None, None, None, None))
        r = (ctypes.c_int64 * (d.value + 1))()
        m = (ctypes.c_int64 * d.value)()
        n = (ctypes.c_int64 * d.value)()
        _check(_lib.qtt_matrix_shape(hv, r, m, n))
        return cls(hv, (list(r), list(m), list(n)))


def qtt_matrix_load(cores, dtypes=("fp64",)):
    """Load host FP64 cores (each of shape (r_prev, m, n, r_next)) onto the device."""
    cores = [np.ascontiguousarray(np.asarray(G, dtype=np.float64)) for G in cores]
    d = len(cores)
    ranks = [cores[0].shape[0]] + [G.shape[3] for G in cores]
    m = [G.shape[1] for G in cores]
    n = [G.shape[2] for G in cores]
    if isinstance(dtypes, (str, int)):
        dtypes = (dtypes,)
    flags = 0
    for t in dtypes:
        flags |= _dtype(t)
    r = (ctypes.c_int64 * (d + 1))(*ranks)
    mm = (ctypes.c_int64 * d)(*m)
    nn = (ctypes.c_int64 * d)(*n)
    ptrs = (ctypes.c_void_p * d)(*[G.ctypes.data for G in cores])
    h = ctypes.c_void_p()
    _check(_lib.qtt_matrix_load(d, r, mm, nn, ptrs, flags, ctypes.byref(h)))
    return QttMatrix(h, (ranks, m, n))


def qtt_matrix_set_diagonals(A, a=0.0, b=None, wc=None):
    """A becomes a I + diag(b) K diag(wc) (b, wc: host FP64 arrays or None)."""
    def host(v):
        if v is None:
            return None, None
        arr = np.ascontiguousarray(v, dtype=np.float64)
        return arr, arr.ctypes.data_as(ctypes.c_void_p)
    bh, bp = host(b)
    wh, wp = host(wc)
    _check(_lib.qtt_matrix_set_diagonals(A.handle, float(a), bp, wp))


def qtt_matrix_info(A):
    d, rows, cols, mr, dt = (ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(),
                             ctypes.c_int64(), ctypes.c_uint32())
    _check(_lib.qtt_matrix_info(A.handle, ctypes.byref(d), ctypes.byref(rows), ctypes.byref(cols),
                                ctypes.byref(mr), ctypes.byref(dt)))
    return {"d": d.value, "rows": rows.value, "cols": cols.value, "max_rank": mr.value,
            "dtypes": dt.value}


def qtt_workspace_bytes(A, compute, nrhs):
    b = ctypes.c_size_t()
    _check(_lib.qtt_workspace_bytes(A.handle, _dtype(compute), int(nrhs), ctypes.byref(b)))
    return b.value


def qtt_solve_workspace_bytes(A, Ainv, inv_compute, nrhs):
    b = ctypes.c_size_t()
    _check(_lib.qtt_solve_workspace_bytes(A.handle, Ainv.handle, _dtype(inv_compute), int(nrhs),
                                          ctypes.byref(b)))
    return b.value


def workspace(nbytes, device="cuda"):
    """Device workspace tensor of at least nbytes (256-byte aligned by the allocator)."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


@_on_stream
def qtt_apply(A, compute, X, Y=None, ws=None, stream=None):
    """Y = A X; returns Y (allocated column-major when not given)."""
    xp, n, k, ldx = _col_major(X, "X")
    if Y is None:
        Y = empty_block(A.rows, k, X.device) if X.dim() == 2 else torch.empty(A.rows, dtype=torch.float64, device=X.device)
    yp, m, ky, ldy = _col_major(Y, "Y")
    if n != A.cols or m != A.rows or ky != k:
        raise ValueError(f"shape mismatch: A is {A.rows}x{A.cols}, X {n}x{k}, Y {m}x{ky}")
    if ws is None:
        ws = workspace(qtt_workspace_bytes(A, compute, k), X.device)
    _check(_lib.qtt_apply(A.handle, _dtype(compute), k, xp, ldx, yp, ldy, ws.data_ptr(),
                          ws.numel() * ws.element_size(), _stream(stream)))
    return Y


def qtt_apply_noalloc(A, compute, X, Y, stream=None):
    """Y = A X through the entry point that allocates nothing (its workspace is
    the library's static device array); X and Y are caller-owned."""
    xp, n, k, ldx = _col_major(X, "X")
    yp, m, ky, ldy = _col_major(Y, "Y")
    if n != A.cols or m != A.rows or ky != k:
        raise ValueError(f"shape mismatch: A is {A.rows}x{A.cols}, X {n}x{k}, Y {m}x{ky}")
    _check(_lib.qtt_apply_noalloc(A.handle, _dtype(compute), k, xp, ldx, yp, ldy, _stream(stream)))
    return Y


@_on_stream
def qtt_apply_batched(A, compute, Xs, Ys=None, ws=None, stream=None):
    """Y_b = A X_b for a list of uneven column-major blocks; returns the list Ys."""
    nb = len(Xs)
    if Ys is None:
        Ys = [empty_block(A.rows, _col_major(X, "X")[2], X.device) for X in Xs]
    xs = [_col_major(X, "X") for X in Xs]
    ys = [_col_major(Y, "Y") for Y in Ys]
    for (xp, n, k, _), (yp, m, ky, _) in zip(xs, ys):
        if n != A.cols or m != A.rows or k != ky:
            raise ValueError("block shape mismatch")
    widths = (ctypes.c_int64 * nb)(*[x[2] for x in xs])
    xptr = (ctypes.c_void_p * nb)(*[x[0] for x in xs])
    ldx = (ctypes.c_int64 * nb)(*[x[3] for x in xs])
    yptr = (ctypes.c_void_p * nb)(*[y[0] for y in ys])
    ldy = (ctypes.c_int64 * nb)(*[y[3] for y in ys])
    if ws is None:
        ws = workspace(qtt_workspace_bytes(A, compute, sum(x[2] for x in xs)), Xs[0].device)
    _check(_lib.qtt_apply_batched(A.handle, _dtype(compute), nb, widths, xptr, ldx, yptr, ldy,
                                  ws.data_ptr(), ws.numel() * ws.element_size(), _stream(stream)))
    return Ys


@_on_stream
def qtt_autotune(A, compute, X, Y, ws, stream=None):
    xp, n, k, ldx = _col_major(X, "X")
    yp, m, _, ldy = _col_major(Y, "Y")
    _check(_lib.qtt_autotune(A.handle, _dtype(compute), k, xp, ldx, yp, ldy, ws.data_ptr(),
                             ws.numel() * ws.element_size(), _stream(stream)))


@_on_stream
def qtt_solve(A, Ainv, inv_compute, F, Sigma=None, rtol=1e-8, max_iter=50, ws=None, stream=None,
              raise_on_fail=True):
    """Refined solve A Sigma = F; returns (Sigma, info, status) with info a list of
    (iters, rel_residual) per column."""
    fp, n, k, ldf = _col_major(F, "F")
    if Sigma is None:
        Sigma = empty_block(n, k, F.device) if F.dim() == 2 else torch.empty(n, dtype=torch.float64, device=F.device)
    sp, _, _, lds = _col_major(Sigma, "Sigma")
    if ws is None:
        ws = workspace(qtt_solve_workspace_bytes(A, Ainv, inv_compute, k), F.device)
    info = (_SolveCol * k)()
    st = _lib.qtt_solve(A.handle, Ainv.handle, _dtype(inv_compute), k, fp, ldf, sp, lds, float(rtol),
                        int(max_iter), ws.data_ptr(), ws.numel() * ws.element_size(), _stream(stream), info)
    if raise_on_fail:
        _check(st)
    else:
        _check(st, allow=(QTT_ERR_NOT_CONVERGED, QTT_ERR_NONFINITE))
    return Sigma, [(c.iters, c.rel_residual) for c in info], st


def _schedule(first, first_compute, first_passes, A_lo, lo_compute, lo_below):
    return _Schedule(first.handle if first is not None else None, _dtype(first_compute or "fp64"), int(first_passes),
                     A_lo.handle if A_lo is not None else None, _dtype(lo_compute or "fp64"), float(lo_below))


def qtt_solve_schedule_workspace_bytes(A, Ainv, inv_compute, nrhs, first=None, first_compute=None, first_passes=0,
                                       A_lo=None, lo_compute=None, lo_below=0.0):
    b = ctypes.c_size_t()
    sc = _schedule(first, first_compute, first_passes, A_lo, lo_compute, lo_below)
    _check(_lib.qtt_solve_schedule_workspace_bytes(A.handle, Ainv.handle, _dtype(inv_compute), ctypes.byref(sc),
                                                   int(nrhs), ctypes.byref(b)))
    return b.value


@_on_stream
def qtt_solve_schedule(A, Ainv, inv_compute, F, Sigma=None, rtol=1e-8, max_iter=50, ws=None, stream=None,
                       first=None, first_compute=None, first_passes=0, A_lo=None, lo_compute=None, lo_below=0.0,
                       raise_on_fail=True):
    """qtt_solve with a schedule: passes 1 .. first_passes apply `first` in
    first_compute (the later ones Ainv in inv_compute), and a pass starting
    with every active column's relative residual <= lo_below updates the
    residual as r -= A_lo dx (A_lo in lo_compute) instead of recomputing it
    in FP64.  Returns (Sigma, info, status) as qtt_solve; info holds the
    computed residuals."""
    fp, n, k, ldf = _col_major(F, "F")
    if Sigma is None:
        Sigma = empty_block(n, k, F.device) if F.dim() == 2 else torch.empty(n, dtype=torch.float64, device=F.device)
    sp, _, _, lds = _col_major(Sigma, "Sigma")
    sc = _schedule(first, first_compute, first_passes, A_lo, lo_compute, lo_below)
    if ws is None:
        ws = workspace(qtt_solve_schedule_workspace_bytes(A, Ainv, inv_compute, k, first, first_compute,
                                                          first_passes, A_lo, lo_compute, lo_below), F.device)
    info = (_SolveCol * k)()
    st = _lib.qtt_solve_schedule(A.handle, Ainv.handle, _dtype(inv_compute), ctypes.byref(sc), k, fp, ldf, sp, lds,
                                 float(rtol), int(max_iter), ws.data_ptr(), ws.numel() * ws.element_size(),
                                 _stream(stream), info)
    if raise_on_fail:
        _check(st)
    else:
        _check(st, allow=(QTT_ERR_NOT_CONVERGED, QTT_ERR_NONFINITE))
    return Sigma, [(c.iters, c.rel_residual) for c in info], st


def qtt_fgmres_workspace_bytes(A, Ainv, inv_compute, nrhs, max_iter):
    n = ctypes.c_size_t()
    _check(_lib.qtt_fgmres_workspace_bytes(A.handle, Ainv.handle if Ainv is not None else None,
                                           _dtype(inv_compute), int(nrhs), int(max_iter), ctypes.byref(n)))
    return n.value


@_on_stream
def qtt_solve_fgmres(A, Ainv, inv_compute, F, Sigma=None, rtol=1e-8, max_iter=30, ws=None, stream=None,
                     raise_on_fail=True):
    """Flexible GMRES solve A Sigma = F, Ainv (or None) the right
    preconditioner; returns (Sigma, info, status) with info a list of
    (steps, relative residual estimate) per column."""
    fp, n, k, ldf = _col_major(F, "F")
    if Sigma is None:
        Sigma = empty_block(n, k, F.device) if F.dim() == 2 else torch.empty(n, dtype=torch.float64, device=F.device)
    sp, _, _, lds = _col_major(Sigma, "Sigma")
    if ws is None:
        ws = workspace(qtt_fgmres_workspace_bytes(A, Ainv, inv_compute, k, max_iter), F.device)
    info = (_SolveCol * k)()
    st = _lib.qtt_solve_fgmres(A.handle, Ainv.handle if Ainv is not None else None, _dtype(inv_compute), k,
                               fp, ldf, sp, lds, float(rtol), int(max_iter), ws.data_ptr(),
                               ws.numel() * ws.element_size(), _stream(stream), info)
    if raise_on_fail:
        _check(st)
    else:
        _check(st, allow=(QTT_ERR_NOT_CONVERGED, QTT_ERR_NONFINITE))
    return Sigma, [(c.iters, c.rel_residual) for c in info], st


def qtt_fgmres_schedule_workspace_bytes(A, Ainv, inv_compute, nrhs, max_iter, first=None, first_compute=None,
                                        first_passes=0, A_lo=None, lo_compute=None, lo_below=0.0):
    n = ctypes.c_size_t()
    sc = _schedule(first, first_compute, first_passes, A_lo, lo_compute, lo_below)
    _check(_lib.qtt_fgmres_schedule_workspace_bytes(A.handle, Ainv.handle if Ainv is not None else None,
                                                    _dtype(inv_compute), ctypes.byref(sc), int(nrhs),
                                                    int(max_iter), ctypes.byref(n)))
    return n.value


@_on_stream
def qtt_solve_fgmres_schedule(A, Ainv, inv_compute, F, Sigma=None, rtol=1e-8, max_iter=30, ws=None, stream=None,
                              first=None, first_compute=None, first_passes=0, A_lo=None, lo_compute=None,
                              lo_below=0.0, raise_on_fail=True):
    """qtt_solve_fgmres with a schedule: steps 1 .. first_passes
    preconditioned with `first` (first_compute), and w = A_lo z_j (lo_compute)
    for a column whose residual estimate before the step is <= lo_below.
    Returns (Sigma, info, status) as qtt_solve_fgmres."""
    fp, n, k, ldf = _col_major(F, "F")
    if Sigma is None:
        Sigma = empty_block(n, k, F.device) if F.dim() == 2 else torch.empty(n, dtype=torch.float64, device=F.device)
    sp, _, _, lds = _col_major(Sigma, "Sigma")
    sc = _schedule(first, first_compute, first_passes, A_lo, lo_compute, lo_below)
    if ws is None:
        ws = workspace(qtt_fgmres_schedule_workspace_bytes(A, Ainv, inv_compute, k, max_iter, first, first_compute,
                                                           first_passes, A_lo, lo_compute, lo_below), F.device)
    info = (_SolveCol * k)()
    st = _lib.qtt_solve_fgmres_schedule(A.handle, Ainv.handle if Ainv is not None else None, _dtype(inv_compute),
                                        ctypes.byref(sc), k, fp, ldf, sp, lds, float(rtol), int(max_iter),
                                        ws.data_ptr(), ws.numel() * ws.element_size(), _stream(stream), info)
    if raise_on_fail:
        _check(st)
    else:
        _check(st, allow=(QTT_ERR_NOT_CONVERGED, QTT_ERR_NONFINITE))
    return Sigma, [(c.iters, c.rel_residual) for c in info], st


@_on_stream
def qtt_matvec_compressed(A, Bcores, Ccores=None, stream=None):
    """Cores of c = A b for a batch of TT vectors (section 4.2).  Bcores[k]:
    contiguous FP64 CUDA tensor (nvec, rb_k, n_k, rb_{k+1}).  Returns the list
    of (nvec, rA_k rb_k, m_k, rA_{k+1} rb_{k+1}) tensors (the merged index is
    alpha + rA beta)."""
    d = len(Bcores)
    nvec = Bcores[0].shape[0]
    rb = [1] + [int(B.shape[3]) for B in Bcores]
    for k, B in enumerate(Bcores):
        if (not B.is_cuda or B.dtype != torch.float64 or not B.is_contiguous() or B.dim() != 4
                or B.shape[0] != nvec or B.shape[1] != rb[k] or B.shape[2] != A.n[k]):
            raise ValueError(f"vector core {k} must be a contiguous FP64 CUDA tensor (nvec, rb_k, n_k, rb_k+1)")
    if Ccores is None:
        Ccores = [torch.empty((nvec, A.ranks[k] * rb[k], A.m[k], A.ranks[k + 1] * rb[k + 1]),
                              dtype=torch.float64, device=Bcores[0].device) for k in range(d)]
    rbh = (ctypes.c_int64 * (d + 1))(*rb)
    bp = (ctypes.c_void_p * d)(*[B.data_ptr() for B in Bcores])
    cp = (ctypes.c_void_p * d)(*[C.data_ptr() for C in Ccores])
    _check(_lib.qtt_matvec_compressed(A.handle, int(nvec), rbh, bp, cp, _stream(stream)))
    return Ccores


@_on_stream
def qtt_solve_fgmres_product(A, M, Y, inv_compute, F, Sigma=None, rtol=1e-8, max_iter=30, ws=None,
                             stream=None, raise_on_fail=True):
    """Flexible GMRES with the product preconditioner z = M (Y v); returns
    (Sigma, info, status)."""
    fp, n, k, ldf = _col_major(F, "F")
    if Sigma is None:
        Sigma = empty_block(n, k, F.device) if F.dim() == 2 else torch.empty(n, dtype=torch.float64, device=F.device)
    sp, _, _, lds = _col_major(Sigma, "Sigma")
    if ws is None:
        ws = workspace(max(qtt_fgmres_workspace_bytes(A, M, inv_compute, k, max_iter),
                           qtt_fgmres_workspace_bytes(A, Y, inv_compute, k, max_iter)), F.device)
    info = (_SolveCol * k)()
    st = _lib.qtt_solve_fgmres_product(A.handle, M.handle, Y.handle, _dtype(inv_compute), k, fp, ldf, sp, lds,
                                       float(rtol), int(max_iter), ws.data_ptr(),
                                       ws.numel() * ws.element_size(), _stream(stream), info)
    if raise_on_fail:
        _check(st)
    else:
        _check(st, allow=(QTT_ERR_NOT_CONVERGED, QTT_ERR_NONFINITE))
    return Sigma, [(c.iters, c.rel_residual) for c in info], st


def qtt_set_shape(A, compute, core, shape):
    _check(_lib.qtt_set_shape(A.handle, _dtype(compute), int(core), int(shape)))


def qtt_use_split_products(A, on=True):
    """Pin (on) or unpin the FP32 split-operand configuration on every interior
    core of A; cores it cannot serve keep the default kernels at launch."""
    for k in range(1, A.d - 1):
        qtt_set_shape(A, "fp32", k, F32_SPLIT if on else -1)
    if not on:
        qtt_set_shape(A, "fp32", -2, 1)     # pinning switched the FP32 pairs off


def qtt_list_shapes(compute):
    ids = (ctypes.c_int32 * 128)()
    n = ctypes.c_int32()
    _check(_lib.qtt_list_shapes(_dtype(compute), ids, 128, ctypes.byref(n)))
    return [ids[i] for i in range(min(n.value, 128))]


def qtt_timing_enable(on=True):
    _check(_lib.qtt_timing_enable(1 if on else 0))


def qtt_timing_reset():
    _check(_lib.qtt_timing_reset())


def qtt_timing_read(compute, position):
    n = ctypes.c_int64()
    ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.qtt_timing_read(_dtype(compute), int(position), ctypes.byref(n), ctypes.byref(ms),
                                ctypes.byref(fl), ctypes.byref(by)))
    return {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}


def qtt_timing_read_shape(compute, shape):
    n = ctypes.c_int64()
    ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.qtt_timing_read_shape(_dtype(compute), int(shape), ctypes.byref(n), ctypes.byref(ms),
                                      ctypes.byref(fl), ctypes.byref(by)))
    return {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}


# ---------------------------------------------------------------- TT form

QTT_ERR_RANK = 9


def _tt_out(n, ranks_cap, device):
    """Output cores with room for ranks up to ranks_cap (d + 1 values)."""
    return [torch.empty(int(ranks_cap[k] * n[k] * ranks_cap[k + 1]), dtype=torch.float64, device=device)
            for k in range(len(n))]


def _tt_result(bufs, n, ranks):
    return [bufs[k][: ranks[k] * n[k] * ranks[k + 1]].view(ranks[k], n[k], ranks[k + 1]) for k in range(len(n))]


@_on_stream
def qtt_tt_round(cores, eps, max_rank=128, seed=1, stream=None, raise_on_cap=True):
    """Round a TT tensor given as a list of (r_{k-1}, n_k, r_k) FP64 CUDA
    tensors; returns (cores, ranks, status)."""
    d = len(cores)
    n = [int(c.shape[1]) for c in cores]
    ranks = [int(cores[0].shape[0])] + [int(c.shape[2]) for c in cores]
    for c in cores:
        if not c.is_cuda or c.dtype != torch.float64 or not c.is_contiguous():
            raise TypeError("TT cores must be contiguous FP64 CUDA tensors")
    cap = [1] + [min(max_rank, r) for r in ranks[1:-1]] + [1]
    out = _tt_out(n, cap, cores[0].device)
    nn = (ctypes.c_int64 * d)(*n)
    rr = (ctypes.c_int64 * (d + 1))(*ranks)
    cin = (ctypes.c_void_p * d)(*[c.data_ptr() for c in cores])
    cout = (ctypes.c_void_p * d)(*[o.data_ptr() for o in out])
    ro = (ctypes.c_int64 * (d + 1))()
    st = _lib.qtt_tt_round(d, nn, rr, cin, float(eps), int(max_rank), int(seed), cout, ro, _stream(stream))
    _check(st, allow=() if raise_on_cap else (QTT_ERR_RANK,))
    r = list(ro)
    return _tt_result(out, n, r), r, st


@_on_stream
def qtt_tt_compress(x, n, eps, max_rank=128, seed=1, stream=None, raise_on_cap=True):
    """TT form of a full FP64 CUDA vector x (length prod n, first digit
    fastest); returns (cores, ranks, status)."""
    d = len(n)
    if not x.is_cuda or x.dtype != torch.float64 or not x.is_contiguous() or x.numel() != int(np.prod(n)):
        raise ValueError("x must be a contiguous FP64 CUDA vector of length prod(n)")
    cap = [1]
    left = 1
    for k in range(d - 1):
        left *= n[k]
        cap.append(min(max_rank, left))
    cap.append(1)
    out = _tt_out(n, cap, x.device)
    nn = (ctypes.c_int64 * d)(*n)
    cout = (ctypes.c_void_p * d)(*[o.data_ptr() for o in out])
    ro = (ctypes.c_int64 * (d + 1))()
    st = _lib.qtt_tt_compress(d, nn, x.data_ptr(), float(eps), int(max_rank), int(seed), cout, ro, _stream(stream))
    _check(st, allow=() if raise_on_cap else (QTT_ERR_RANK,))
    r = list(ro)
    return _tt_result(out, n, r), r, st


def qtt_matrix_cores(A):
    """The handle's FP64 cores as host numpy arrays (r, m, n, r')."""
    out = [np.empty((A.ranks[k], A.m[k], A.n[k], A.ranks[k + 1])) for k in range(A.d)]
    ptrs = (ctypes.c_void_p * A.d)(*[o.ctypes.data for o in out])
    _check(_lib.qtt_matrix_cores(A.handle, ptrs))
    return out


@_on_stream
def qtt_invert_newton_schulz(A, X0, eps, max_rank=128, max_iter=12, tol=0.0, theta=0.0, seed=1,
                             dtypes=("fp64",), stream=None, raise_on_cap=True):
    """Newton-Hotelling-Schulz inverse of A from X0; returns (handle,
    history, steps, status)."""
    flags = 0
    for t in dtypes:
        flags |= DTYPES[t]
    out = ctypes.c_void_p()
    hist = (ctypes.c_double * (max_iter + 1))()
    steps = ctypes.c_int32()
    st = _lib.qtt_invert_newton_schulz(A.handle, X0.handle, float(eps), int(max_rank), int(max_iter), float(tol),
                                       float(theta), int(seed), flags, ctypes.byref(out), hist, ctypes.byref(steps),
                                       _stream(stream))
    _check(st, allow=() if raise_on_cap else (QTT_ERR_RANK,))
    X = QttMatrix._from_handle(out.value)
    return X, list(hist)[: steps.value + 1], steps.value, st
