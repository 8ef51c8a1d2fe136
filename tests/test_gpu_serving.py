"""GPU: captured sweeps, uneven batching at full size, and the continuous-
batching server (each result the same alone and in the mix)."""
import numpy as np
import pytest

from oracle import qtt_oracle as O
from paper_1511_06029_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1511_06029_amd import qtt
    return qtt


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_graph_replays_follow_new_data(Q):
    """The first call launches directly and captures; later calls with the
    same pointers replay the graph and must read the new input data."""
    cores = I.gaussian_qtt([1, 6, 9, 5, 1], [8] * 4, seed=3)
    A = Q.qtt_matrix_load(cores, dtypes=("fp64", "bf16"))
    X = Q.empty_block(4096, 3)
    Y = Q.empty_block(4096, 3)
    ws = Q.workspace(Q.qtt_workspace_bytes(A, "fp64", 3))
    for rep in range(4):
        Xh = I.rhs(4096, 3, seed=100 + rep)
        X.copy_(Q.to_block(Xh))
        Y.zero_()
        torch.cuda.synchronize()
        Q.qtt_apply(A, "fp64", X, Y, ws=ws)
        torch.cuda.synchronize()
        assert rel(Y.cpu().numpy(), O.qtt_apply_alg2(cores, Xh)) < 1e-12, rep
    # the replayed result is bitwise the direct one
    Xh = I.rhs(4096, 3, seed=7)
    X.copy_(Q.to_block(Xh))
    Q.qtt_apply(A, "bf16", X, Y, ws=ws)
    first = Y.cpu().numpy().copy()
    for _ in range(3):
        Y.zero_()
        Q.qtt_apply(A, "bf16", X, Y, ws=ws)
        assert np.array_equal(Y.cpu().numpy(), first)
    A.free()


def _wave_capacity(Q, A, dtype, ws_bytes):
    """Vectors per wave: the largest w with qtt_workspace_bytes(w) <= ws_bytes
    (the rule the library applies to a caller's workspace)."""
    lo, hi = 1, 1
    while Q.qtt_workspace_bytes(A, dtype, hi * 2) <= ws_bytes:
        hi *= 2
    hi *= 2
    while lo < hi - 1:
        mid = (lo + hi) // 2
        if Q.qtt_workspace_bytes(A, dtype, mid) <= ws_bytes:
            lo = mid
        else:
            hi = mid
    return lo


@pytest.mark.slow
def test_batched_uneven_L7_fp32(Q):
    """64 blocks of widths drawn from {1,2,4,8,16,32} against the L=7 operator in
    FP32, through one apply_batched call.  Every column is compared with the
    FP64 apply of the same column (itself pinned to the oracle), and the first
    and last column of every workspace wave are checked by the oracle."""
    w = I.WORKLOADS["batched_L7"]
    Ac, _ = I.perturbed_identity_pair(w["ranks"], [8] * 7, seed=w["core_seed"])
    widths = I.uneven_widths(w["nblocks"], seed=w["width_seed"])
    A = Q.qtt_matrix_load(Ac, dtypes=("fp32", "fp64"))
    N = 8 ** 7
    g = torch.Generator(device="cuda").manual_seed(w["rhs_seed"])
    Xs = [torch.randn((wd, N), generator=g, device="cuda", dtype=torch.float64).t() for wd in widths]
    ws_bytes = min(Q.qtt_workspace_bytes(A, "fp32", sum(widths)), 64 * 2 ** 30)
    ws = Q.workspace(ws_bytes)
    Ys = Q.qtt_apply_batched(A, "fp32", Xs, ws=ws)
    torch.cuda.synchronize()
    del ws
    # every column against the FP64 sweep
    ws64 = Q.workspace(Q.qtt_workspace_bytes(A, "fp64", 32))
    worst = 0.0
    for b, (X, Y) in enumerate(zip(Xs, Ys)):
        R = Q.qtt_apply(A, "fp64", X, ws=ws64)
        err = ((Y - R).norm(dim=0) / R.norm(dim=0)).max().item()
        worst = max(worst, err)
        assert err < 1e-5, (b, err)
    del ws64
    # the oracle on the first and last column of each wave
    cap = _wave_capacity(Q, A, "fp32", ws_bytes)
    total = sum(widths)
    starts = np.cumsum([0] + widths)
    cols = sorted({g0 for g0 in range(0, total, cap)} | {min(g0 + cap, total) - 1 for g0 in range(0, total, cap)})
    print(f"{len(widths)} blocks, {total} vectors, {cap} per wave; FP32 vs FP64 worst {worst:.2e}; "
          f"oracle on columns {cols}")
    for gcol in cols:
        b = int(np.searchsorted(starts, gcol, side="right") - 1)
        c = gcol - int(starts[b])
        x = Xs[b][:, c].cpu().numpy()
        ref = O.qtt_apply_alg2(Ac, x)
        assert rel(Ys[b][:, c].cpu().numpy(), ref) < 1e-5, (gcol, b, c)
    A.free()


def _ops():
    ops = {}
    for t, (name, ranks) in enumerate((("op0", [1, 6, 8, 6, 1]), ("op1", [1, 5, 5, 1]),
                                       ("op2", [1, 8, 8, 8, 1]))):
        L = len(ranks) - 1
        ops[name] = I.perturbed_identity_pair(ranks, [8] * L, seed=700 + t)
    return ops


@pytest.mark.parametrize("lo", [None, "fp32"])
def test_server_alone_equals_mix(Q, lo):
    """Every result of a mixed run is bitwise the same request served alone,
    and the oracle's FP64 residual of each column is <= 1e-8; also with the
    late residual updates by an FP32 copy of A (decided per column, so the
    mix cannot change a column's route)."""
    from paper_1511_06029_amd.serving import Request, SolveServer
    kw = dict(residual_lo=lo, lo_below=1e-4) if lo else {}
    ops = _ops()
    g = I.rng(5)
    spec = []
    for i in range(12):
        op = f"op{int(g.integers(3))}"
        k = int(g.integers(1, 4))
        N = 8 ** (len(ops[op][0]))
        spec.append((i, op, I.rhs(N, k, seed=500 + i)))

    def make():
        return [Request(rid=i, op=op, F=Q.to_block(F)) for i, op, F in spec]

    # mixed: everything waiting at once, two slots
    srv = SolveServer(ops, inv_dtype="bf16", budget_bytes=2 * 10 ** 9, n_slots=2, **kw)
    mixed = make()
    torch.cuda.synchronize()
    stats = srv.run_trace(mixed, realtime=False)
    srv.close()
    assert stats["all_converged"]
    assert stats["batches"] < len(mixed)          # requests were coalesced
    # alone: one slot, one request at a time
    srv = SolveServer(ops, inv_dtype="bf16", budget_bytes=2 * 10 ** 9, n_slots=1, **kw)
    for r in make():
        torch.cuda.synchronize()
        srv.run_trace([r], realtime=False)
        m = mixed[r.rid]
        assert np.array_equal(r.Sigma.cpu().numpy(), m.Sigma.cpu().numpy()), r.rid
        F = spec[r.rid][2]
        Ac = ops[r.op][0]
        res = F - O.qtt_apply_alg2(Ac, m.Sigma.cpu().numpy().reshape(F.shape))
        assert np.all(np.linalg.norm(res, axis=0) <= 1e-8 * np.linalg.norm(F, axis=0) * 1.0001)
    srv.close()


@pytest.mark.slow
def test_server_alone_equals_mix_serving_shapes(Q):
    """The serving workload's operator shapes (mode 8, L = 5, 6 and 7, ranks
    between 16 and 32, requests of 1 to 16 vectors): every result of a mixed
    run with three slots is bitwise the result of the same request served
    alone, and the oracle's FP64 residual of each is <= 1e-8 (L = 5 and 6:
    every column; L = 7: the first column of each request)."""
    from paper_1511_06029_amd.serving import Request, SolveServer
    shapes = (("L5r17", 5, 17), ("L6r29", 6, 29), ("L7r24", 7, 24))
    ops = {name: I.perturbed_identity_pair([1] + [r] * (L - 1) + [1], [8] * L, seed=740 + t)
           for t, (name, L, r) in enumerate(shapes)}
    g = I.rng(77)
    spec = []
    for i in range(10):
        name, L, _ = shapes[int(g.integers(3))]
        spec.append((i, name, I.rhs(8 ** L, int(g.integers(1, 17)), seed=760 + i)))

    def make():
        return [Request(rid=i, op=op, F=Q.to_block(F)) for i, op, F in spec]

    srv = SolveServer(ops, inv_dtype="bf16", budget_bytes=60 * 10 ** 9, n_slots=3)
    mixed = make()
    torch.cuda.synchronize()
    stats = srv.run_trace(mixed, realtime=False)
    srv.close()
    assert stats["all_converged"]
    assert stats["batches"] < len(mixed)
    srv = SolveServer(ops, inv_dtype="bf16", budget_bytes=60 * 10 ** 9, n_slots=1)
    for r in make():
        torch.cuda.synchronize()
        srv.run_trace([r], realtime=False)
        m = mixed[r.rid]
        assert np.array_equal(r.Sigma.cpu().numpy(), m.Sigma.cpu().numpy()), r.rid
        F = spec[r.rid][2]
        S = m.Sigma.cpu().numpy().reshape(F.shape)
        cols = [0] if F.shape[0] == 8 ** 7 else list(range(F.shape[1]))
        Ac = ops[r.op][0]
        res = F[:, cols] - O.qtt_apply_alg2(Ac, S[:, cols])
        assert np.all(np.linalg.norm(res, axis=0) <= 1e-8 * np.linalg.norm(F[:, cols], axis=0) * 1.0001), r.rid
        r.Sigma = None
        m.Sigma = None
    srv.close()


def test_server_budget_serialises_batches(Q):
    """With a budget that holds one batch at a time, batches never overlap."""
    from paper_1511_06029_amd.serving import Request, SolveServer
    ops = _ops()
    one = {"op0": ops["op0"]}
    srv0 = SolveServer(one, inv_dtype="fp32", budget_bytes=10 ** 9, n_slots=1)
    need = srv0.batch_bytes("op0", 2)
    srv0.close()
    srv = SolveServer(one, inv_dtype="fp32", budget_bytes=int(need * 1.5), n_slots=3, max_batch_rhs=2)
    reqs = [Request(rid=i, op="op0", F=Q.to_block(I.rhs(4096, 2, seed=900 + i))) for i in range(4)]
    torch.cuda.synchronize()
    stats = srv.run_trace(reqs, realtime=False)
    srv.close()
    assert stats["all_converged"] and stats["batches"] == 4
    spans = sorted((a, d) for _, _, _, a, d in srv.log)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0 - 1e-6


def test_autotune_keeps_parity(Q):
    """The autotuner times every configuration per core and keeps the fastest;
    the tuned sweep still matches the oracle, and its choice survives (the
    next apply is bitwise the autotuner's own result)."""
    cores = I.gaussian_qtt([1, 16, 32, 32, 16, 1], [8] * 5, seed=61)
    X = I.rhs(8 ** 5, 4, seed=62)
    ref = O.qtt_apply_alg2(cores, X)
    A = Q.qtt_matrix_load(cores, dtypes=("fp64", "bf16"))
    Xd = Q.to_block(X)
    for dt, tol in (("fp64", 1e-12), ("bf16", 3e-2)):
        Y = Q.empty_block(8 ** 5, 4)
        ws = Q.workspace(Q.qtt_workspace_bytes(A, dt, 4))
        Q.qtt_autotune(A, dt, Xd, Y, ws)
        tuned = Y.cpu().numpy()
        assert rel(tuned, ref) < tol
        again = Q.qtt_apply(A, dt, Xd, ws=ws).cpu().numpy()
        assert np.array_equal(again, tuned)
    A.free()
