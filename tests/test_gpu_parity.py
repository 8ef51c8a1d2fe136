"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (normwise per column, worst column):
  FP64 sweep  1e-12, and elementwise |y - y_ref| <= 1e-12 max|y_ref|
  FP32 sweep  1e-5
  BF16 sweep  3e-2 for the Gaussian-core operators (8 significant bits:
              unit roundoff 2^-8; d roundings of cores and intermediates of
              random sign add up to about sqrt(2d/3) 2^-8 ~ 0.01 at d = 7);
              the refined solve then restores 1e-8.
FP32 and BF16 are also checked entry by entry against the rounding bound
|Y - A X| <= gamma (|A| |X|) of parity_bounds (|A| with cores |G_k|, applied
by the oracle), and block by block (512 consecutive entries of a column) at
the normwise tolerance, so an error confined to one tile is seen.
  refined solve: relative residual <= 1e-8 recomputed by the oracle.
Integer-exact cases (identity, permutation cores) are bitwise.
"""
import numpy as np
import pytest

from oracle import qtt_oracle as O
from paper_1511_06029_amd import inputs as I
import parity_bounds as B
import qtt_structures as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 3e-2, "fp32s": 1e-4}


@pytest.fixture(scope="module")
def Q():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1511_06029_amd import qtt
    return qtt


def colrel(Y, R):
    Y = np.asarray(Y).reshape(R.shape[0], -1)
    R = R.reshape(R.shape[0], -1)
    return max(np.linalg.norm(Y[:, c] - R[:, c]) / max(np.linalg.norm(R[:, c]), 1e-300)
               for c in range(R.shape[1]))


def elementwise_ok(Y, R, tol):
    Y = np.asarray(Y).reshape(R.shape[0], -1)
    R = R.reshape(R.shape[0], -1)
    scale = np.abs(R).max(axis=0)
    return np.all(np.abs(Y - R) <= tol * scale[None, :])


def check_reduced(Y, ref, cores, X, dtype, label):
    """Element-wise rounding bound and block-wise tolerance for FP32/BF16;
    prints the measured errors."""
    ratio = B.elementwise_ratio(Y, ref, cores, X, dtype)
    blk = B.blockwise_rel(Y, ref)
    print(f"{label} {dtype}: normwise {colrel(Y, ref):.3e}, blockwise {blk:.3e}, "
          f"elementwise error / bound {ratio:.3f}")
    assert ratio <= 1.0, (label, ratio)
    assert blk <= TOL[dtype], (label, blk)


def gpu_apply(Q, cores, X, dtype, ws_nrhs=None):
    A = Q.qtt_matrix_load(cores, dtypes=(dtype,))
    Xd = Q.to_block(X)
    ws = None
    if ws_nrhs is not None:
        ws = Q.workspace(Q.qtt_workspace_bytes(A, dtype, ws_nrhs))
    Y = Q.qtt_apply(A, dtype, Xd, ws=ws)
    torch.cuda.synchronize()
    out = Y.cpu().numpy()
    A.free()
    return out


# ------------------------------------------------------------------ exact cases

@pytest.mark.parametrize("dtype", ["fp64", "fp32", "bf16"])
def test_identity_bitwise(Q, dtype):
    X = I.rhs(8 ** 3, 3, seed=1)
    if dtype != "fp64":   # values exactly representable in the compute type
        X = np.round(X * 8) / 8
    Y = gpu_apply(Q, I.identity_qtt([8] * 3), X, dtype)
    assert np.array_equal(Y, X)


def test_permutation_bitwise_fp64(Q):
    g = I.rng(9)
    mats = [np.eye(8)[g.permutation(8)] for _ in range(4)]
    X = I.rhs(8 ** 4, 2, seed=3)
    Y = gpu_apply(Q, S.kron_cores(mats), X, "fp64")
    assert np.array_equal(Y, S.modewise_apply(mats, X))


# ------------------------------------------------------------------ random operators

SHAPES = [
    ("octree_L4", [1, 7, 9, 6, 1], [8] * 4, [8] * 4),
    ("rect_uneven", [1, 3, 5, 2, 1], [2, 3, 4, 2], [3, 2, 2, 4]),
    ("single_core", [1, 1], [5], [3]),
    ("unit_modes", [1, 2, 1], [1, 4], [3, 1]),
    ("shape_example", [1, 4, 4, 1], [4, 2, 2], [4, 2, 2]),
    ("rank40_L3", [1, 40, 40, 1], [8] * 3, [8] * 3),
    ("L2_small_C", [1, 16, 1], [8, 8], [8, 8]),
]


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("name,ranks,m,n", SHAPES, ids=[s[0] for s in SHAPES])
def test_random_shapes(Q, name, ranks, m, n, dtype):
    cores = I.gaussian_qtt(ranks, m, n, seed=11)
    N = int(np.prod(n))
    X = I.rhs(N, 3, seed=12)
    ref = O.qtt_apply_alg2(cores, X)
    Y = gpu_apply(Q, cores, X, dtype)
    err = colrel(Y, ref)
    print(f"{name} {dtype} rel err {err:.3e}")
    assert err <= TOL[dtype]
    if dtype == "fp64":
        assert elementwise_ok(Y, ref, 1e-12)
    else:
        check_reduced(Y, ref, cores, X, dtype, name)


@pytest.mark.parametrize("K", [1, 16])
@pytest.mark.parametrize("dtype", ["fp64", "fp32", "bf16"])
def test_synthetic_L6(Q, K, dtype):
    """L=6 (N=262144), ranks [1,16,32,32,32,16,1], Gaussian cores scaled
    1/sqrt(8 r_{k-1}), K=1 and K=16 seeded N(0,1) right-hand sides."""
    w = I.WORKLOADS["synthetic_L6"]
    cores = I.gaussian_qtt(w["ranks"], [8] * 6, seed=w["core_seed"])
    X = I.rhs(8 ** 6, K, seed=w["rhs_seed"])
    ref = O.qtt_apply_alg2(cores, X)
    Y = gpu_apply(Q, cores, X, dtype)
    err = colrel(Y, ref)
    print(f"L6 K={K} {dtype} rel err {err:.3e}")
    assert err <= TOL[dtype]
    if dtype == "fp64":
        assert elementwise_ok(Y, ref, 1e-12)
    else:
        check_reduced(Y, ref, cores, X, dtype, f"L6 K={K}")
    if dtype == "fp64":
        assert elementwise_ok(Y, ref, 1e-12)


def test_volume_L4_fp64(Q):
    """Volume operator on the 16^3 grid (Morton order, octree digits), TT-SVD at
    1e-10: ranks [1,27,173,27,1] (non-power-of-two rank, several row tiles)."""
    A = O.volume_matrix(4)
    cores, _ = O.qtt_matrix_from_dense(A, [8] * 4, [8] * 4, 1e-10)
    assert [G.shape[3] for G in cores] == [27, 173, 27, 1]
    X = I.rhs(4096, 1, seed=I.WORKLOADS["volume_L4"]["rhs_seed"])
    ref = O.qtt_apply_alg2(cores, X)
    Y = gpu_apply(Q, cores, X, "fp64")
    assert colrel(Y, ref) <= 1e-12 and elementwise_ok(Y, ref, 1e-12)
    assert colrel(Y, A @ X) <= 1e-9      # within the compression error of A itself


# ------------------------------------------------------------------ layouts, waves, batching

def test_padded_ld_and_waves(Q):
    cores = I.gaussian_qtt([1, 6, 12, 5, 1], [8] * 4, seed=21)
    X = I.rhs(4096, 5, seed=22)
    ref = O.qtt_apply_alg2(cores, X)
    A = Q.qtt_matrix_load(cores, dtypes=("fp64",))
    Xp = torch.zeros((5, 4100), dtype=torch.float64, device="cuda")
    Xp[:, :4096] = torch.from_numpy(X.T.copy()).cuda()
    Xv = Xp.t()[:4096]                       # ld = 4100
    Yp = torch.full((5, 4098), 7.0, dtype=torch.float64, device="cuda")
    Yv = Yp.t()[:4096]                       # ld = 4098
    ws = Q.workspace(Q.qtt_workspace_bytes(A, "fp64", 1))   # one vector per wave
    Q.qtt_apply(A, "fp64", Xv, Yv, ws=ws)
    torch.cuda.synchronize()
    Yh = Yp.cpu().numpy()
    assert np.all(Yh[:, 4096:] == 7.0)       # padding untouched
    assert colrel(Yh[:, :4096].T, ref) <= 1e-12
    A.free()


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_batched_uneven(Q, dtype):
    cores = I.gaussian_qtt([1, 8, 16, 8, 1], [8] * 4, seed=31)
    widths = [1, 4, 2, 0, 7, 1, 3]
    A = Q.qtt_matrix_load(cores, dtypes=(dtype,))
    Xs_h = [I.rhs(4096, w, seed=40 + b) for b, w in enumerate(widths)]
    Xs = [Q.to_block(x) if x.shape[1] else Q.empty_block(4096, 0) for x in Xs_h]
    total = sum(widths)
    for ws_n in (total, 3):                  # one wave, then several waves
        ws = Q.workspace(Q.qtt_workspace_bytes(A, dtype, ws_n))
        Ys = Q.qtt_apply_batched(A, dtype, Xs, ws=ws)
        torch.cuda.synchronize()
        for x, y in zip(Xs_h, Ys):
            if x.shape[1]:
                assert colrel(y.cpu().numpy(), O.qtt_apply_alg2(cores, x)) <= TOL[dtype]
    A.free()


def test_batched_matches_single_bitwise(Q):
    """Batch invariance: a vector's result does not depend on its batch."""
    cores = I.gaussian_qtt([1, 8, 16, 8, 1], [8] * 4, seed=33)
    A = Q.qtt_matrix_load(cores, dtypes=("fp64", "bf16"))
    X = I.rhs(4096, 6, seed=34)
    for dt in ("fp64", "bf16"):
        alone = [Q.qtt_apply(A, dt, Q.to_block(X[:, c])).cpu().numpy() for c in range(6)]
        Ys = Q.qtt_apply_batched(A, dt, [Q.to_block(X[:, :2]), Q.to_block(X[:, 2:])])
        mixed = np.concatenate([y.cpu().numpy() for y in Ys], axis=1)
        for c in range(6):
            assert np.array_equal(mixed[:, c], alone[c])
    A.free()


# ------------------------------------------------------------------ solve

@pytest.mark.parametrize("inv", ["fp64", "fp32", "bf16"])
def test_solve_L4_vs_dense(Q, inv):
    ranks = [1, 6, 8, 6, 1]
    Ac, Aic = I.perturbed_identity_pair(ranks, [8] * 4, seed=81)
    F = I.rhs(4096, 3, seed=82)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    Ai = Q.qtt_matrix_load(Aic, dtypes=(inv,))
    Sig, info, st = Q.qtt_solve(A, Ai, inv, Q.to_block(F), rtol=1e-8)
    Sh = Sig.cpu().numpy()
    ref = np.linalg.solve(O.qtt_to_dense(Ac), F)
    res = F - O.qtt_apply_alg2(Ac, Sh)
    for c in range(3):
        assert np.linalg.norm(res[:, c]) <= 1e-8 * np.linalg.norm(F[:, c]) * 1.0001
        assert info[c][1] <= 1e-8
    assert colrel(Sh, ref) <= 3e-8
    A.free()
    Ai.free()


def test_solve_iterations_match_oracle_fp64(Q):
    ranks = [1, 6, 8, 6, 1]
    Ac, Aic = I.perturbed_identity_pair(ranks, [8] * 4, seed=83)
    F = I.rhs(4096, 2, seed=84)
    Xo, hist = O.richardson_solve(Ac, Aic, F, rtol=1e-8)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    Ai = Q.qtt_matrix_load(Aic, dtypes=("fp64",))
    Sig, info, st = Q.qtt_solve(A, Ai, "fp64", Q.to_block(F), rtol=1e-8)
    assert [c[0] for c in info] == [len(hist)] * 2
    assert colrel(Sig.cpu().numpy(), Xo) <= 1e-12
    A.free()
    Ai.free()


@pytest.mark.slow
def test_refine_L7_full_size(Q):
    """The refined solve at full size: L=7 (N=2,097,152), ranks
    [1,24,32,32,32,32,24,1], K=8; the oracle recomputes the relative residual of
    two sampled columns, and checks one FP64 A apply elementwise."""
    w = I.WORKLOADS["refine_L7"]
    Ac, Aic = I.perturbed_identity_pair(w["ranks"], [8] * 7, seed=w["core_seed"], eps=w["eps"])
    F = I.rhs(8 ** 7, w["K"], seed=w["rhs_seed"])
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    Ai = Q.qtt_matrix_load(Aic, dtypes=("bf16", "fp64"))
    Fd = Q.to_block(F)
    Sig, info, st = Q.qtt_solve(A, Ai, "bf16", Fd, rtol=w["rtol"])
    Sh = Sig.cpu().numpy()
    for c in (0, w["K"] - 1):
        r = F[:, c] - O.qtt_apply_alg2(Ac, Sh[:, c])
        assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(F[:, c]) * 1.0001
    Y = Q.qtt_apply(A, "fp64", Q.to_block(F[:, :1]))
    ref = O.qtt_apply_alg2(Ac, F[:, :1])
    assert colrel(Y.cpu().numpy(), ref) <= 1e-12 and elementwise_ok(Y.cpu().numpy(), ref, 1e-12)
    A.free()
    Ai.free()


# ------------------------------------------------------------------ errors

def test_error_paths(Q):
    cores = I.gaussian_qtt([1, 3, 1], [8, 8], seed=5)
    A = Q.qtt_matrix_load(cores, dtypes=("fp64",))
    X = Q.to_block(I.rhs(64, 2, seed=1))
    with pytest.raises(Q.QttError) as e:
        Q.qtt_apply(A, "bf16", X)            # dtype not loaded
    assert e.value.status == 8
    with pytest.raises(Q.QttError) as e:
        Q.qtt_apply(A, "fp64", X, X)         # output overlaps input
    assert e.value.status == 1
    with pytest.raises(Q.QttError) as e:
        Q.qtt_apply(A, "fp64", X, ws=Q.workspace(16))
    assert e.value.status == 7
    Ai = Q.qtt_matrix_load([-G for G in cores], dtypes=("fp64",))
    Sig, info, st = Q.qtt_solve(A, Ai, "fp64", X, max_iter=3, raise_on_fail=False)
    assert st == 5                            # not a contraction: not converged
    A.free()
    Ai.free()


@pytest.mark.parametrize("inv", ["fp64", "bf16", "fp32s"])
def test_nonfinite_rhs_reported(Q, inv):
    """A NaN or an infinity in one column of F makes its residual norm
    non-finite: qtt_solve and qtt_solve_fgmres return QTT_ERR_NONFINITE (6)
    instead of iterating, and the finite columns are still solved.  fp32s:
    the FP32 inverse with split-product cores (core 2 here; an infinity
    splits into a NaN low part, still non-finite)."""
    Ac, Aic = I.perturbed_identity_pair([1, 6, 8, 6, 1], [8] * 4, seed=95)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    if inv == "fp32s":
        Ai = Q.qtt_matrix_load(Aic, dtypes=("fp32",))
        Q.qtt_use_split_products(Ai)
        inv = "fp32"
    else:
        Ai = Q.qtt_matrix_load(Aic, dtypes=("fp64", "bf16"))
    for bad in (np.nan, np.inf):
        F = I.rhs(4096, 3, seed=96)
        F[17, 1] = bad
        Sig, info, st = Q.qtt_solve(A, Ai, inv, Q.to_block(F), rtol=1e-8, raise_on_fail=False)
        assert st == 6, (bad, st)
        assert not np.isfinite(info[1][1])
        S = Sig.cpu().numpy()
        for c in (0, 2):
            res = F[:, c] - O.qtt_apply_alg2(Ac, S[:, c])
            assert np.linalg.norm(res) <= 1e-8 * np.linalg.norm(F[:, c]) * 1.0001, (bad, c)
        Sig, info, st = Q.qtt_solve_fgmres(A, Ai, inv, Q.to_block(F), rtol=1e-8, raise_on_fail=False)
        assert st == 6, (bad, st)
    A.free()
    Ai.free()


def test_nonfinite_rhs_reported_scheduled(Q):
    """The scheduled solvers (BF16 inverse in the first pass or step, FP32
    after it, late residual updates by an FP32 copy of A) report a NaN or an
    infinity in one column as QTT_ERR_NONFINITE and still solve the finite
    columns to the tolerance (the oracle recomputes their residuals)."""
    Ac, Aic = I.perturbed_identity_pair([1, 6, 8, 6, 1], [8] * 4, seed=95)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    Alo = Q.qtt_matrix_load(Ac, dtypes=("fp32",))
    Ai = Q.qtt_matrix_load(Aic, dtypes=("fp32", "bf16"))
    sched = dict(first=Ai, first_compute="bf16", first_passes=1, A_lo=Alo, lo_compute="fp32", lo_below=1e-4)
    for bad in (np.nan, np.inf):
        F = I.rhs(4096, 3, seed=96)
        F[17, 1] = bad
        for solve in (Q.qtt_solve_schedule, Q.qtt_solve_fgmres_schedule):
            Sig, info, st = solve(A, Ai, "fp32", Q.to_block(F), rtol=1e-8, raise_on_fail=False, **sched)
            assert st == 6, (bad, st, solve.__name__)
            assert not np.isfinite(info[1][1])
            S = Sig.cpu().numpy()
            for c in (0, 2):
                res = F[:, c] - O.qtt_apply_alg2(Ac, S[:, c])
                assert np.linalg.norm(res) <= 1e-8 * np.linalg.norm(F[:, c]) * 1.0001, (bad, c, solve.__name__)
    for h in (A, Alo, Ai):
        h.free()


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "bf16"])
def test_every_kernel_configuration(Q, dtype):
    """Pin each kernel configuration on every core in turn (a configuration
    that cannot serve a core falls back to the default) and compare with the
    oracle: covers the single-operand, streamed, 4x4x4, register-resident,
    direct-to-LDS and vector-ALU variants."""
    cases = [([1, 24, 32, 32, 24, 1], 3), ([1, 16, 32, 16, 1], 2), ([1, 9, 13, 1], 2)]
    for ranks, K in cases:
        L = len(ranks) - 1
        cores = I.gaussian_qtt(ranks, [8] * L, seed=17 + L)
        X = I.rhs(8 ** L, K, seed=18 + L)
        ref = O.qtt_apply_alg2(cores, X)
        mag = B.magnitude(cores, X)
        A = Q.qtt_matrix_load(cores, dtypes=(dtype,))
        Xd = Q.to_block(X)
        for shape in Q.qtt_list_shapes(dtype):
            for k in range(L):
                Q.qtt_set_shape(A, dtype, k, shape)
            Y = Q.qtt_apply(A, dtype, Xd)
            torch.cuda.synchronize()
            err = colrel(Y.cpu().numpy(), ref)
            assert err <= TOL[dtype], (ranks, shape, err)
            if dtype == "fp64":
                assert elementwise_ok(Y.cpu().numpy(), ref, 1e-12), (ranks, shape)
            else:
                assert B.elementwise_ratio(Y.cpu().numpy(), ref, cores, X, dtype, mag) <= 1.0, (ranks, shape)
                assert B.blockwise_rel(Y.cpu().numpy(), ref) <= TOL[dtype], (ranks, shape)
        A.free()


def test_fp32_split_products(Q):
    """FP32 sweeps with the split-operand configuration pinned on the interior
    cores, against the oracle: element-wise within the split's rounding bound,
    block-wise within 1e-4.  The cases cover 256, 192, 128 and 64 rows (all
    four store counts), K_in of 104 (a partial last step), 128, 192 and 256, a
    core it cannot serve (r_k = 13: the default kernels run there), one to
    four tiles per workgroup (one or two peeled tiles, the loop, its odd tail), and
    the launch timing shows which cores ran it."""
    cases = [([1, 24, 32, 32, 24, 1], 7, 3), ([1, 16, 32, 16, 1], 2, 2), ([1, 8, 13, 8, 1], 3, 1),
             ([1, 24, 32, 24, 1], 24, 2)]
    for ranks, K, n_split in cases:
        L = len(ranks) - 1
        cores = I.gaussian_qtt(ranks, [8] * L, seed=41 + L + K)
        X = I.rhs(8 ** L, K, seed=42 + L + K)
        ref = O.qtt_apply_alg2(cores, X)
        A = Q.qtt_matrix_load(cores, dtypes=("fp32",))
        Q.qtt_use_split_products(A)
        Xd = Q.to_block(X)
        Q.qtt_apply(A, "fp32", Xd)
        torch.cuda.synchronize()
        Q.qtt_timing_reset()
        Q.qtt_timing_enable(True)
        Y = Q.qtt_apply(A, "fp32", Xd)
        torch.cuda.synchronize()
        Q.qtt_timing_enable(False)
        ran = Q.qtt_timing_read_shape("fp32", Q.F32_SPLIT)["launches"]
        Q.qtt_timing_reset()
        assert ran == n_split, (ranks, ran)
        check_reduced(Y.cpu().numpy(), ref, cores, X, "fp32s", f"split {ranks} K={K}")
        # pinned on the first and last cores too, which it cannot serve: the
        # defaults run there
        Q.qtt_set_shape(A, "fp32", 0, Q.F32_SPLIT)
        Q.qtt_set_shape(A, "fp32", L - 1, Q.F32_SPLIT)
        Y = Q.qtt_apply(A, "fp32", Xd)
        torch.cuda.synchronize()
        check_reduced(Y.cpu().numpy(), ref, cores, X, "fp32s", f"split, all cores pinned, {ranks} K={K}")
        # unpinned: the default FP32 kernels again, at FP32's own bound
        Q.qtt_use_split_products(A, False)
        Y = Q.qtt_apply(A, "fp32", Xd)
        torch.cuda.synchronize()
        check_reduced(Y.cpu().numpy(), ref, cores, X, "fp32", f"unpinned {ranks} K={K}")
        A.free()


def test_fp32_split_batched_uneven(Q):
    """The split-product configuration on uneven blocks (several segments for
    the first and last cores, one or several workspace waves), each block
    against the oracle within the split's bound, and a block's bits the same
    alone and in the batch."""
    ranks = [1, 24, 32, 32, 24, 1]
    cores = I.gaussian_qtt(ranks, [8] * 5, seed=51)
    widths = [1, 4, 2, 0, 7, 1, 3]
    A = Q.qtt_matrix_load(cores, dtypes=("fp32",))
    Q.qtt_use_split_products(A)
    Xs_h = [I.rhs(8 ** 5, w, seed=60 + b) for b, w in enumerate(widths)]
    Xs = [Q.to_block(x) if x.shape[1] else Q.empty_block(8 ** 5, 0) for x in Xs_h]
    total = sum(widths)
    for ws_n in (total, 3):
        ws = Q.workspace(Q.qtt_workspace_bytes(A, "fp32", ws_n))
        Ys = Q.qtt_apply_batched(A, "fp32", Xs, ws=ws)
        torch.cuda.synchronize()
        for b, (x, y) in enumerate(zip(Xs_h, Ys)):
            if x.shape[1]:
                check_reduced(y.cpu().numpy(), O.qtt_apply_alg2(cores, x), cores, x, "fp32s",
                              f"split batched block {b} (workspace {ws_n} vectors)")
    alone = Q.qtt_apply(A, "fp32", Xs[4])
    torch.cuda.synchronize()
    assert np.array_equal(alone.cpu().numpy(), Ys[4].cpu().numpy())
    A.free()


def test_solve_schedule(Q):
    """qtt_solve_schedule.  With no schedule it is qtt_solve, and with more
    first passes than the solve needs it is qtt_solve with the first inverse
    (same bits either way).  A BF16 first pass and split-product (or plain,
    from the same handle) FP32 passes after it converge to the tolerance,
    the residual recomputed by the oracle.  Residual updates with a split
    FP32 copy of A in the late passes: the computed residual stays within
    1e-10 of the true one (recomputed in FP64), lo_below = 0 changes no bit,
    and a first pass with the update gives qtt_solve's first iterate.  Bad
    schedules are rejected."""
    Ac, Aic = I.perturbed_identity_pair([1, 8, 16, 16, 8, 1], [8] * 5, seed=97)
    F = I.rhs(8 ** 5, 3, seed=98)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    As = Q.qtt_matrix_load(Ac, dtypes=("fp32",))
    Q.qtt_use_split_products(As)
    Ai = Q.qtt_matrix_load(Aic, dtypes=("bf16", "fp32"))
    Ais = Q.qtt_matrix_load(Aic, dtypes=("fp32",))
    Q.qtt_use_split_products(Ais)
    Fd = Q.to_block(F)
    Fn = np.linalg.norm(F, axis=0)

    def true_rel(S):
        Sh = S.cpu().numpy()
        return np.array([np.linalg.norm(F[:, c] - O.qtt_apply_alg2(Ac, Sh[:, c])) / Fn[c] for c in range(3)])

    S0, info0, _ = Q.qtt_solve(A, Ais, "fp32", Fd, rtol=1e-8)
    S1, info1, _ = Q.qtt_solve_schedule(A, Ais, "fp32", Fd, rtol=1e-8)
    assert np.array_equal(S0.cpu().numpy(), S1.cpu().numpy()) and info0 == info1
    S2, info2, _ = Q.qtt_solve_schedule(A, Ais, "fp32", Fd, rtol=1e-8, first=Ai, first_compute="bf16",
                                        first_passes=1)
    print("schedule passes", [c[0] for c in info2], "split only", [c[0] for c in info0])
    assert np.all(true_rel(S2) <= 1e-8 * 1.0001)
    # every pass within the first ones: qtt_solve with the first inverse
    S3, info3, _ = Q.qtt_solve(A, Ai, "bf16", Fd, rtol=1e-8)
    S4, info4, _ = Q.qtt_solve_schedule(A, Ais, "fp32", Fd, rtol=1e-8, first=Ai, first_compute="bf16",
                                        first_passes=50)
    assert np.array_equal(S3.cpu().numpy(), S4.cpu().numpy()) and info3 == info4
    # one handle holding both copies, plain FP32 arithmetic after the first pass
    S5, _, _ = Q.qtt_solve_schedule(A, Ai, "fp32", Fd, rtol=1e-8, first=Ai, first_compute="bf16", first_passes=1)
    assert np.all(true_rel(S5) <= 1e-8 * 1.0001)
    # residual updates with A's split FP32 copy once every column is below 1e-5
    sched = dict(first=Ai, first_compute="bf16", first_passes=1, A_lo=As, lo_compute="fp32")
    S6, info6, _ = Q.qtt_solve_schedule(A, Ais, "fp32", Fd, rtol=1e-8, lo_below=1e-5, **sched)
    t6 = true_rel(S6)
    print("updated residuals", [c for c in info6], "true", t6)
    assert np.all(np.abs(t6 - np.array([c[1] for c in info6])) <= 1e-10)
    assert np.all(t6 <= 1e-8 * 1.0001)
    assert [c[0] for c in info6] == [c[0] for c in info2]
    S7, info7, _ = Q.qtt_solve_schedule(A, Ais, "fp32", Fd, rtol=1e-8, lo_below=0.0, **sched)
    assert np.array_equal(S7.cpu().numpy(), S2.cpu().numpy()) and info7 == info2
    # the update from the first pass on: sigma_1 = Ainv F as qtt_solve's, and
    # the computed residual within the split apply's error of the true one
    S8, info8, _ = Q.qtt_solve_schedule(A, Ais, "fp32", Fd, rtol=1e-8, max_iter=1, lo_below=2.0, A_lo=As,
                                        lo_compute="fp32", raise_on_fail=False)
    S9, info9, _ = Q.qtt_solve(A, Ais, "fp32", Fd, rtol=1e-8, max_iter=1, raise_on_fail=False)
    assert np.array_equal(S8.cpu().numpy(), S9.cpu().numpy())
    assert np.all(np.abs(np.array([c[1] for c in info8]) - np.array([c[1] for c in info9])) <= 1e-4)
    for bad in (dict(first_passes=-1, first=Ai, first_compute="bf16"), dict(first_passes=1),
                dict(A_lo=As, lo_compute="fp32", lo_below=-1.0), dict(A_lo=As, lo_compute="bf16", lo_below=1e-5)):
        with pytest.raises(Q.QttError):
            Q.qtt_solve_schedule(A, Ais, "fp32", Fd, rtol=1e-8, ws=Q.workspace(1 << 30), **bad)
    for h in (A, As, Ai, Ais):
        h.free()


@pytest.mark.slow
def test_refine_L7_split_fp32_inverse(Q):
    """The reported solve in the benchmark's launch configuration: L=7, K=8,
    the inverse computed on the GPU by Newton-Hotelling-Schulz from the
    first-order inverse (ranks held at 32, the benchmark's call), its FP32
    copy applied with the split-product configuration on every interior core.
    Three passes; the oracle recomputes the relative residual of two sampled
    columns, and one inverse apply is checked element by element against the
    oracle's apply of the same cores within the split's rounding bound.  The
    schedule with the inverse's BF16 copy in the first pass also takes three
    passes, with and without residual updates by A's split FP32 copy in the
    late passes; every column's true residual (FP64 apply) is within 1e-10 of
    the computed one and below the tolerance."""
    w = I.WORKLOADS["refine_L7"]
    Ac, Aic = I.perturbed_identity_pair(w["ranks"], [8] * 7, seed=w["core_seed"], eps=w["eps"])
    F = I.rhs(8 ** 7, w["K"], seed=w["rhs_seed"])
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    Ai0 = Q.qtt_matrix_load(Aic, dtypes=("fp64", "fp32", "bf16"))
    Ai, hist, steps, _ = Q.qtt_invert_newton_schulz(A, Ai0, 1e-10, max_rank=32, max_iter=6, theta=0.1, seed=5,
                                                     dtypes=("fp64", "fp32", "bf16"), raise_on_cap=False)
    cores = Q.qtt_matrix_cores(Ai)
    Ais = Q.qtt_matrix_load(cores, dtypes=("fp32",))
    Q.qtt_use_split_products(Ais)
    Sig, info, st = Q.qtt_solve(A, Ais, "fp32", Q.to_block(F), rtol=w["rtol"])
    print("split fp32 inverse passes", [c[0] for c in info], "residuals", [c[1] for c in info])
    assert [c[0] for c in info] == [3] * w["K"]
    Sh = Sig.cpu().numpy()
    for c in (0, w["K"] - 1):
        r = F[:, c] - O.qtt_apply_alg2(Ac, Sh[:, c])
        assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(F[:, c]) * 1.0001
    Y = Q.qtt_apply(Ais, "fp32", Q.to_block(F[:, :1]))
    torch.cuda.synchronize()
    ref = O.qtt_apply_alg2(cores, F[:, :1])
    check_reduced(Y.cpu().numpy(), ref, cores, F[:, :1], "fp32s", "split inverse apply, L=7")
    # the schedule with the BF16 copy of the same inverse in the first pass,
    # then also with the residual updated by A's split FP32 copy once every
    # column is below 1e-5 (the benchmark's call)
    As = Q.qtt_matrix_load(Ac, dtypes=("fp32",))
    Q.qtt_use_split_products(As)
    Fd = Q.to_block(F)
    for lo in (None, As):
        Sig, info, st = Q.qtt_solve_schedule(A, Ais, "fp32", Fd, rtol=w["rtol"], first=Ai, first_compute="bf16",
                                             first_passes=1, A_lo=lo, lo_compute="fp32", lo_below=1e-5)
        print("schedule passes", [c[0] for c in info], "residuals", [c[1] for c in info])
        assert [c[0] for c in info] == [3] * w["K"]
        # the true residual of every column, A applied in FP64 on the GPU
        R = Fd - Q.qtt_apply(A, "fp64", Sig)
        true = (torch.linalg.vector_norm(R, dim=0) / torch.linalg.vector_norm(Fd, dim=0)).cpu().numpy()
        print("true residuals", true)
        assert np.all(np.abs(true - np.array([c[1] for c in info])) <= 1e-10)
        assert np.all(true <= 1e-8 * 1.0001)
        Sh = Sig.cpu().numpy()
        for c in (0, w["K"] - 1):
            r = F[:, c] - O.qtt_apply_alg2(Ac, Sh[:, c])
            assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(F[:, c]) * 1.0001
    for h in (A, As, Ai0, Ai, Ais):
        h.free()


def test_timing_by_configuration(Q):
    """Launch timing summed by kernel configuration partitions the sums by
    core position: same launches, same flops, and the default configurations
    are the ones recorded (fused FP64 core pairs, the vector-ALU last core;
    the first core's short-contraction kernel for BF16)."""
    ranks = [1, 24, 32, 32, 24, 1]
    cores = I.gaussian_qtt(ranks, [8] * 5, seed=81)
    X = I.rhs(8 ** 5, 2, seed=82)
    A = Q.qtt_matrix_load(cores, dtypes=("fp64", "bf16"))
    Xd = Q.to_block(X)
    for dt in ("fp64", "bf16"):
        Q.qtt_apply(A, dt, Xd)          # first call: direct launches, graph capture
        torch.cuda.synchronize()
        Q.qtt_timing_reset()
        Q.qtt_timing_enable(True)
        Q.qtt_apply(A, dt, Xd)
        torch.cuda.synchronize()
        Q.qtt_timing_enable(False)
        by_pos = [Q.qtt_timing_read(dt, p) for p in range(4)]
        by_shape = {sh: Q.qtt_timing_read_shape(dt, sh) for sh in Q.qtt_list_shapes(dt) + Q.PAIR_SHAPES}
        Q.qtt_timing_reset()
        used = {sh: r for sh, r in by_shape.items() if r["launches"]}
        assert sum(r["launches"] for r in by_pos) == sum(r["launches"] for r in used.values())
        # 2 R_out K_in flops per column, C_k = 8^4 columns per vector, 2 vectors
        flops = sum(2.0 * c.shape[0] * c.shape[3] * c.shape[1] * c.shape[2] for c in cores) * 8 ** 4 * 2
        assert np.isclose(sum(r["flops"] for r in by_pos), sum(r["flops"] for r in used.values()))
        assert np.isclose(sum(r["flops"] for r in used.values()), flops)
        assert all(r["ms"] > 0 for r in used.values())
        if dt == "fp64":
            # fused pairs (0, 1): first core, r_1 = 24, 256 rows next; (2, 3): r_3 = 32,
            # 192 rows next; then the last core on the vector ALUs (K_in = 192: the
            # whole-line configuration 49)
            assert set(used) == {90 + 4 + 0 + 1, 90 + 0 + 2 + 0, 49}, used.keys()
            assert sum(r["launches"] for r in used.values()) == 3
        else:
            assert 34 in used and sum(r["launches"] for r in used.values()) == len(ranks) - 1, used.keys()
    assert Q.qtt_timing_read_shape("fp64", 9999)["launches"] == 0
    A.free()


@pytest.mark.parametrize("dtype,base", [("fp64", 90), ("fp32", 100)])
def test_fused_pairs_any_rank(Q, dtype, base):
    """The fused pair kernels at boundary ranks other than 24 and 32 (padded
    rows and contraction): the first core with r_1 = 20 and an interior pair
    with r_3 = 29, against the oracle and against the sweep with pairs
    switched off; and a refined solve through them."""
    ranks = [1, 20, 29, 29, 20, 1]
    cores = I.gaussian_qtt(ranks, [8] * 5, seed=91)
    X = I.rhs(8 ** 5, 3, seed=92)
    ref = O.qtt_apply_alg2(cores, X)
    A = Q.qtt_matrix_load(cores, dtypes=(dtype,))
    Xd = Q.to_block(X)
    Q.qtt_timing_reset()
    Q.qtt_timing_enable(True)
    Yp = Q.qtt_apply(A, dtype, Xd).cpu().numpy()
    torch.cuda.synchronize()
    Q.qtt_timing_enable(False)
    used = {sh for sh in Q.PAIR_SHAPES if Q.qtt_timing_read_shape(dtype, sh)["launches"]}
    Q.qtt_timing_reset()
    assert used == {base + 4 + 2 + 1, base + 0 + 2 + 0}, used   # (0,1) padded, 232 rows next; (2,3) padded, 160 rows
    tol = TOL[dtype]
    assert colrel(Yp, ref) <= tol and elementwise_ok(Yp, ref, tol)
    Q.qtt_set_shape(A, dtype, -2, 0)
    Ys = Q.qtt_apply(A, dtype, Xd).cpu().numpy()
    assert colrel(Ys, ref) <= tol
    assert colrel(Yp, Ys) <= tol / 10
    Q.qtt_set_shape(A, dtype, -2, 1)
    A.free()
    # a refined solve through the fused pairs (FP64 residual, this dtype's inverse)
    Ac, Aic = I.perturbed_identity_pair(ranks, [8] * 5, seed=93)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    Ai = Q.qtt_matrix_load(Aic, dtypes=(dtype,))
    F = I.rhs(8 ** 5, 2, seed=94)
    Sig, info, st = Q.qtt_solve(A, Ai, dtype, Q.to_block(F), rtol=1e-8)
    assert st == 0 and all(c[1] <= 1e-8 for c in info)
    S = Sig.cpu().numpy().reshape(F.shape)
    res = F - O.qtt_apply_alg2(Ac, S)
    assert np.all(np.linalg.norm(res, axis=0) <= 1e-8 * np.linalg.norm(F, axis=0) * 1.0001)
    A.free()
    Ai.free()


@pytest.mark.slow
def test_apply_and_solve_L8_maximum_size(Q):
    """The largest operator of the serving trace: L=8 (N=16,777,216), ranks
    [1,24,32,32,32,32,32,24,1] (three fused pairs, a single interior core,
    the last core).  FP64 apply of two vectors against the oracle (first
    column, normwise and elementwise), and a refined solve with the BF16
    inverse whose residual the oracle recomputes (second column)."""
    ranks = [1, 24, 32, 32, 32, 32, 32, 24, 1]
    Ac, Aic = I.perturbed_identity_pair(ranks, [8] * 8, seed=51, eps=0.1)
    X = I.rhs(8 ** 8, 2, seed=52)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    Ai = Q.qtt_matrix_load(Aic, dtypes=("bf16",))
    Xd = Q.to_block(X)
    Y = Q.qtt_apply(A, "fp64", Xd).cpu().numpy()
    ref = O.qtt_apply_alg2(Ac, X[:, :1])
    assert colrel(Y[:, :1], ref) <= 1e-12 and elementwise_ok(Y[:, :1], ref, 1e-12)
    del Y, ref
    Sig, info, st = Q.qtt_solve(A, Ai, "bf16", Xd, rtol=1e-8)
    s1 = Sig[:, 1].cpu().numpy()
    r = X[:, 1] - O.qtt_apply_alg2(Ac, s1[:, None])[:, 0]
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(X[:, 1]) * 1.0001
    assert info[1][1] == pytest.approx(np.linalg.norm(r) / np.linalg.norm(X[:, 1]), rel=1e-3)
    A.free()
    Ai.free()


def _bf16_rne(x):
    """Round-to-nearest-even of float32(x) to BF16, by integer arithmetic on
    the float32 bits (ties to even), returned as FP64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _bf16_of_double(x):
    """Nearest-even BF16 of each FP64 value, by exact rational arithmetic
    (Python's round() of a Fraction breaks ties to even); returned as FP64.
    Normal BF16 range only."""
    from fractions import Fraction
    import math
    out = np.empty(len(x))
    for t, v in enumerate(np.asarray(x, dtype=np.float64)):
        if v == 0.0:
            out[t] = v
            continue
        _, e = math.frexp(v)                    # |v| = m 2^e, 1/2 <= m < 1
        step = Fraction(2) ** (e - 8)           # 8 significant bits
        out[t] = float(round(Fraction(v) / step) * step)
    return out


def test_bf16_rounding_from_fp64_is_single(Q):
    """FP64 inputs just beside a BF16 tie (the tie plus or minus a few FP64
    units, far below FP32's resolution): rounding through FP32 first would
    land on the tie and break it to even; the first core rounds once, so the
    BF16 identity returns the nearest BF16 of each FP64 value."""
    g = I.rng(962)
    hi = (g.integers(0x0080, 0x7F00, 2048).astype(np.uint32) | (g.integers(0, 2, 2048).astype(np.uint32) << 15)) << 16
    ties = (hi | 0x8000).view(np.float32).astype(np.float64)
    ulp = np.abs(ties) * 2.0 ** -45
    vals = np.concatenate([ties + ulp, ties - ulp, ties * (1 + 2.0 ** -40), ties * (1 - 2.0 ** -40), ties])
    N = 512
    n_col = len(vals) // N
    X = vals[: N * n_col].reshape(N, n_col, order="F")
    E = _bf16_of_double(X.reshape(-1, order="F")).reshape(X.shape, order="F")
    # the inputs do separate single from double rounding
    assert np.count_nonzero(E != _bf16_rne(X)) > N
    A = Q.qtt_matrix_load(I.identity_qtt([8] * 3), dtypes=("bf16",))
    Y = Q.qtt_apply(A, "bf16", Q.to_block(X)).cpu().numpy()
    assert np.array_equal(Y, E)
    A.free()
    # the loader rounds core values once too: a scalar core with value v
    for v in (float(ties[0] + ulp[0]), float(ties[1] - ulp[1])):
        core = [np.full((1, 1, 1, 1), v)]
        B = Q.qtt_matrix_load(core, dtypes=("bf16",))
        y = Q.qtt_apply(B, "bf16", Q.to_block(np.ones((1, 1)))).cpu().numpy()
        assert y[0, 0] == _bf16_of_double(np.array([v]))[0], v
        B.free()


def test_bf16_rounding_bitwise_through_identity(Q):
    """A BF16 identity operator rounds its input once (to BF16, nearest even)
    and carries it exactly, so its output equals that rounding bit for bit:
    exact ties with even and odd upper bits, values just below and above a
    tie, the largest finite BF16 range, and random values.  (Infinities are
    left out: the identity core's zeros would turn them into NaN; so are
    subnormals, which the matrix cores may flush.)"""
    g = I.rng(961)
    hi = (g.integers(0x0080, 0x7F7F, 4096).astype(np.uint32) | (g.integers(0, 2, 4096).astype(np.uint32) << 15)) << 16
    ties = (hi | 0x8000).view(np.float32)
    near = (hi | 0x7FFF).view(np.float32)
    above = (hi | 0x8001).view(np.float32)
    edge = np.array([3.38e38, -3.38e38, 1.0, -1.0, 0.0], dtype=np.float32)
    rnd = g.standard_normal(4096).astype(np.float32)
    vals = np.concatenate([ties, near, above, edge, rnd])
    N = 512
    n_col = len(vals) // N
    X = vals[: N * n_col].astype(np.float64).reshape(N, n_col, order="F")
    A = Q.qtt_matrix_load(I.identity_qtt([8] * 3), dtypes=("bf16",))
    Y = Q.qtt_apply(A, "bf16", Q.to_block(X)).cpu().numpy()
    E = _bf16_rne(X)
    assert np.all(np.isfinite(E))
    assert np.array_equal(Y, E)
    A.free()
