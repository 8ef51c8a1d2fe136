"""GPU: TT rounding, compression of a full vector, the compressed "QTT
solve" chain (compress, compressed product, round) and the Newton-Schulz
inversion, against the oracle.

Rounded cores are not unique (any orthonormal basis of the kept subspaces
serves), so the comparison is on what is: the represented tensor (expanded,
within eps ||c||, the bound Algorithm 1 guarantees) and the ranks (equal to
the oracle's where the singular values leave a clear gap at the threshold).
The GPU sketch is random (Philox4x32-10 normals); the oracle's rounding is
the deterministic definition.
"""
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


def _rand_tt(ranks, modes, seed, scale=1.0):
    """Gaussian cores; the first one scaled (the tensor scales by `scale`)."""
    g = I.rng(seed)
    return [(scale if k == 0 else 1.0) * g.standard_normal((ranks[k], modes[k], ranks[k + 1]))
            for k in range(len(modes))]


def _tt_sum(a, b):
    d = len(a)
    out = []
    for k in range(d):
        x, y = a[k], b[k]
        if k == 0:
            out.append(np.concatenate([x, y], axis=2))
        elif k == d - 1:
            out.append(np.concatenate([x, y], axis=0))
        else:
            G = np.zeros((x.shape[0] + y.shape[0], x.shape[1], x.shape[2] + y.shape[2]))
            G[:x.shape[0], :, :x.shape[2]] = x
            G[x.shape[0]:, :, x.shape[2]:] = y
            out.append(G)
    return out


def _dev(cores):
    return [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in cores]


def _host(cores):
    return [c.cpu().numpy() for c in cores]


def _right_orthonormal(cores, atol=1e-7):
    """Cores 2..d with orthonormal rows, to the accuracy the truncation gives:
    a row scaled by 1/s_j carries a relative error of about the unit roundoff
    times s_max / s_j (1e-9 for singular values near 1e-7 ||c||)."""
    for G in cores[1:]:
        M = G.reshape(G.shape[0], -1)
        if not np.allclose(M @ M.T, np.eye(G.shape[0]), atol=atol):
            return False
    return True


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-9])
def test_round_matches_oracle(Q, eps):
    """A sum of a large TT and one 1e-6 times smaller (ranks 6..8 + 5..7, so
    the ranks at a cut have a clear gap at 1e-2 and 1e-4, where the small term
    goes, and at 1e-9, where it stays) rounded at eps: the oracle rounding's
    ranks, the same tensor within eps ||c||, and the GPU result within eps ||c||
    of c."""
    modes = [8, 6, 8, 6, 8]
    big = _rand_tt([1, 6, 8, 8, 6, 1], modes, seed=31)
    small = _rand_tt([1, 5, 7, 7, 5, 1], modes, seed=32, scale=1e-6)
    c = _tt_sum(big, small)
    v = O.tt_full(c)
    ref, _ = O.tt_round(c, eps)
    cores, ranks, st = Q.qtt_tt_round(_dev(c), eps, seed=5)
    got = _host(cores)
    w = O.tt_full(got)
    print(f"eps {eps}: GPU ranks {ranks}, oracle {[1] + [G.shape[2] for G in ref]}, "
          f"error {np.linalg.norm(w - v) / np.linalg.norm(v):.3e}")
    assert ranks == [1] + [G.shape[2] for G in ref]
    assert np.linalg.norm(w - v) <= eps * np.linalg.norm(v) * 1.01
    assert np.linalg.norm(w - O.tt_full(ref)) <= 2 * eps * np.linalg.norm(v)
    assert _right_orthonormal(got)


def test_round_exact_rank_recovery(Q):
    """a + a (ranks doubled) rounds back to a's ranks and the value 2a, to
    rounding accuracy."""
    a = _rand_tt([1, 7, 12, 6, 1], [8, 8, 8, 8], seed=33)
    c = _tt_sum(a, a)
    cores, ranks, _ = Q.qtt_tt_round(_dev(c), 1e-12, seed=6)
    ref = 2 * O.tt_full(a)
    assert ranks == [1, 7, 12, 6, 1]
    assert np.linalg.norm(O.tt_full(_host(cores)) - ref) <= 1e-11 * np.linalg.norm(ref)


def test_round_compressed_product(Q):
    """The compressed product of section 4.2 (ranks multiply: 24 x 4 = 96) of
    a QTT matrix and a TT vector, rounded on the GPU: the result equals the
    oracle's apply of the matrix to the expanded vector within eps, with the
    oracle rounding's ranks."""
    Ac, _ = I.perturbed_identity_pair([1, 24, 24, 24, 1], [8] * 4, seed=34)
    b = _rand_tt([1, 4, 4, 4, 1], [8] * 4, seed=35)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    B = [torch.from_numpy(np.ascontiguousarray(G[None])).cuda() for G in b]
    C = Q.qtt_matvec_compressed(A, B)
    prod = [Cc[0].contiguous() for Cc in C]
    assert [int(P.shape[2]) for P in prod[:-1]] == [96, 96, 96]
    eps = 1e-9
    cores, ranks, _ = Q.qtt_tt_round(prod, eps, seed=7)
    y = O.qtt_apply_alg2(Ac, O.tt_full(b))
    w = O.tt_full(_host(cores))
    ref, _ = O.tt_round([P.cpu().numpy() for P in prod], eps)
    print(f"product ranks 96 -> GPU {ranks}, oracle {[1] + [G.shape[2] for G in ref]}")
    assert ranks == [1] + [G.shape[2] for G in ref]
    assert np.linalg.norm(w - y) <= eps * np.linalg.norm(y) * 1.01 + 1e-13 * np.linalg.norm(y)
    A.free()


@pytest.mark.parametrize("L,eps", [(3, 1e-10), (4, 1e-6), (5, 1e-6), (5, 1e-10)])
def test_compress_diric_matches_oracle(Q, L, eps):
    """Section 5.1's right-hand side f = phi(x) phi(y) phi(z) on the (2^L)^3
    grid in octree order, compressed on the GPU: the oracle TT-SVD's ranks and
    an error within eps ||f||."""
    f = O.diric_rhs(L)
    ref, _ = O.tt_svd(f.reshape((8,) * L, order="F"), eps)
    x = torch.from_numpy(f).cuda()
    cores, ranks, _ = Q.qtt_tt_compress(x, [8] * L, eps, seed=8)
    w = O.tt_full(_host(cores))
    err = np.linalg.norm(w - f) / np.linalg.norm(f)
    print(f"L={L} eps={eps}: GPU ranks {ranks}, oracle {[1] + [G.shape[2] for G in ref]}, error {err:.3e}")
    assert ranks == [1] + [G.shape[2] for G in ref]
    assert err <= eps * 1.01


def test_qtt_solve_chain(Q):
    """The "QTT solve" of section 5.2 on the GPU: compress f (diric), the
    compressed product with the compressed inverse (ranks multiply), round.
    The result is the inverse applied to f (the oracle's full-vector apply)
    within the two tolerances."""
    L = 4
    _, Aic = I.perturbed_identity_pair([1, 8, 8, 8, 1], [8] * L, seed=36)
    f = O.diric_rhs(L)
    eps_c, eps_r = 1e-8, 1e-8
    Ai = Q.qtt_matrix_load(Aic, dtypes=("fp64",))
    fc, fr, _ = Q.qtt_tt_compress(torch.from_numpy(f).cuda(), [8] * L, eps_c, seed=9)
    C = Q.qtt_matvec_compressed(Ai, [G[None].contiguous() for G in fc])
    prod = [Cc[0].contiguous() for Cc in C]
    cores, ranks, _ = Q.qtt_tt_round(prod, eps_r, seed=10)
    y = O.qtt_apply_alg2(Aic, f)
    w = O.tt_full(_host(cores))
    err = np.linalg.norm(w - y) / np.linalg.norm(y)
    print(f"QTT solve L=4: f ranks {fr}, product ranks {[1] + [int(P.shape[2]) for P in prod]}, "
          f"rounded {ranks}, error {err:.3e}")
    assert err <= 3 * (eps_c + eps_r)
    Ai.free()


@pytest.mark.parametrize("ranks,modes", [([1, 3, 4, 4, 3, 1], [2] * 5), ([1, 4, 1], [8, 8])])
def test_newton_schulz_matches_oracle(Q, ranks, modes):
    """Newton-Hotelling-Schulz from the first-order inverse, no truncation
    (eps = 1e-14): the GPU's residual history and final inverse follow the
    oracle's iteration, and the inverse is inv(A)."""
    Ac, Aic = I.perturbed_identity_pair(ranks, modes, seed=37)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    X0 = Q.qtt_matrix_load(Aic, dtypes=("fp64",))
    X, hist, steps, _ = Q.qtt_invert_newton_schulz(A, X0, 1e-14, max_iter=4, seed=11)
    Xo, hist_o = O.newton_schulz(Ac, Aic, 1e-14, max_iter=4)
    print(f"GPU history {hist}, oracle {hist_o}")
    assert steps == len(hist_o) - 1
    assert np.allclose(hist, hist_o, rtol=1e-4, atol=1e-12)
    Xg = O.qtt_to_dense(Q.qtt_matrix_cores(X))
    Ad = O.qtt_to_dense(Ac)
    Ainv = np.linalg.inv(Ad)
    assert np.linalg.norm(Xg - O.qtt_to_dense(Xo)) <= 1e-10 * np.linalg.norm(Ainv)
    assert np.linalg.norm(Xg - Ainv) <= 1e-10 * np.linalg.norm(Ainv)
    for G in (A, X0, X):
        G.free()


def test_newton_schulz_L4_feeds_solve(Q):
    """L=4 operator of ranks 8 (N = 4096), eps = 1e-7, adaptive rounding of
    the early iterates (theta = 0.1): the residual squares
    down to the rounding level, the inverse matches inv(A) to that level, and
    a refined solve with it (BF16) converges to 1e-8 in fewer passes than with
    the first-order inverse it started from."""
    Ac, Aic = I.perturbed_identity_pair([1, 8, 8, 8, 1], [8] * 4, seed=38)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    X0 = Q.qtt_matrix_load(Aic, dtypes=("fp64", "bf16"))
    X, hist, steps, _ = Q.qtt_invert_newton_schulz(A, X0, 1e-7, max_iter=8, tol=1e-6, theta=0.1, seed=12,
                                                   dtypes=("fp64", "bf16"))
    print(f"history {hist}, ranks {X.ranks}")
    assert hist[-1] <= 1e-5
    for h0, h1 in zip(hist[:2], hist[1:3]):
        assert h1 <= 64.0 * h0 ** 2 + 1e-7        # ||R^2||_F <= ||R||_F^2 (norms / sqrt(N))
    Ad = O.qtt_to_dense(Ac)
    Ainv = np.linalg.inv(Ad)
    Xg = O.qtt_to_dense(Q.qtt_matrix_cores(X))
    assert np.linalg.norm(Xg - Ainv) <= 1e-5 * np.linalg.norm(Ainv)
    F = I.rhs(4096, 2, seed=39)
    _, info_ns, _ = Q.qtt_solve(A, X, "bf16", Q.to_block(F), rtol=1e-8)
    _, info_0, _ = Q.qtt_solve(A, X0, "bf16", Q.to_block(F), rtol=1e-8)
    print(f"passes with the Newton-Schulz inverse {[c[0] for c in info_ns]}, first-order {[c[0] for c in info_0]}")
    assert max(c[0] for c in info_ns) < max(c[0] for c in info_0)
    for G in (A, X0, X):
        G.free()


def test_tt_errors(Q):
    c = _dev(_rand_tt([1, 3, 1], [4, 4], seed=40))
    with pytest.raises(Q.QttError):
        Q.qtt_tt_round(c, -1.0)
    with pytest.raises(Q.QttError):
        Q.qtt_tt_round(c, 1e-6, max_rank=0)
    with pytest.raises(Q.QttError):
        Q.qtt_tt_round(c, 1e-6, max_rank=129)
    # a tolerance needing rank 16 at a cap of 8: the best at 8 and QTT_ERR_RANK
    a = _rand_tt([1, 16, 16, 1], [16, 16, 16], seed=41)
    cores, ranks, st = Q.qtt_tt_round(_dev(a), 1e-12, max_rank=8, raise_on_cap=False)
    assert st == Q.QTT_ERR_RANK and max(ranks) <= 8


def test_newton_schulz_adaptive_matches_oracle(Q):
    """The adaptive rule (theta = 0.1) at eps = 1e-9 on the mode-2 operator:
    the GPU's iterate ranks and residual history follow the oracle's."""
    Ac, Aic = I.perturbed_identity_pair([1, 3, 4, 4, 3, 1], [2] * 5, seed=15)
    A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
    X0 = Q.qtt_matrix_load(Aic, dtypes=("fp64",))
    X, hist, steps, _ = Q.qtt_invert_newton_schulz(A, X0, 1e-9, max_iter=6, theta=0.1, seed=13)
    Xo, hist_o = O.newton_schulz(Ac, Aic, 1e-9, max_iter=6, theta=0.1)
    print(f"GPU {hist} ranks {X.ranks}; oracle {hist_o} ranks {[1] + [G.shape[3] for G in Xo]}")
    assert X.ranks == [1] + [G.shape[3] for G in Xo]
    assert np.allclose(hist, hist_o, rtol=1e-3, atol=1e-9)
    Ainv = np.linalg.inv(O.qtt_to_dense(Ac))
    assert np.linalg.norm(O.qtt_to_dense(Q.qtt_matrix_cores(X)) - Ainv) <= 1e-7 * np.linalg.norm(Ainv)
    for G in (A, X0, X):
        G.free()
