"""Pins of the oracle's TT rounding, the section 5.2 right-hand side, the QTT
matrix product and sum, and the Newton-Hotelling-Schulz inversion, against
facts that do not come from those functions: the dense TT-SVD (itself pinned
to Eckart-Young), exact rank recovery, the rounding error bound, the
Dirichlet-kernel sum of cosines, dense products, and the dense iteration.
"""
import numpy as np
import pytest

from oracle import qtt_oracle as O
from paper_1511_06029_amd import inputs as I


def _rand_tt(ranks, modes, seed, scale=1.0):
    g = I.rng(seed)
    return [scale * g.standard_normal((ranks[k], modes[k], ranks[k + 1])) for k in range(len(modes))]


def _tt_sum(a, b):
    """Cores of a + b (TT sum, written out independently of qtt_lincomb)."""
    d = len(a)
    out = []
    for k in range(d):
        x, y = a[k], b[k]
        n = x.shape[1]
        if d == 1:
            out.append(x + y)
        elif k == 0:
            out.append(np.concatenate([x, y], axis=2))
        elif k == d - 1:
            out.append(np.concatenate([x, y], axis=0))
        else:
            G = np.zeros((x.shape[0] + y.shape[0], n, x.shape[2] + y.shape[2]))
            G[:x.shape[0], :, :x.shape[2]] = x
            G[x.shape[0]:, :, x.shape[2]:] = y
            out.append(G)
    return out


def test_tt_full_matches_entries():
    c = _rand_tt([1, 2, 3, 1], [3, 2, 4], seed=1)
    v = O.tt_full(c)
    for i1 in range(3):
        for i2 in range(2):
            for i3 in range(4):
                e = (c[0][:, i1, :] @ c[1][:, i2, :] @ c[2][:, i3, :])[0, 0]
                assert v[i1 + 3 * (i2 + 2 * i3)] == pytest.approx(e, rel=1e-14, abs=1e-14)


def test_round_recovers_exact_ranks():
    """a + a has twice a's ranks and rounds back to a's ranks (generic cores),
    with the value 2a."""
    a = _rand_tt([1, 3, 4, 2, 1], [3, 4, 2, 5], seed=2)
    c = _tt_sum(a, a)
    assert [G.shape[2] for G in c[:-1]] == [6, 8, 4]
    r, tails = O.tt_round(c, 1e-12)
    assert [G.shape[2] for G in r[:-1]] == [3, 4, 2]
    ref = 2 * O.tt_full(a)
    assert np.linalg.norm(O.tt_full(r) - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("eps", [1e-1, 1e-3, 1e-6])
def test_round_equals_dense_ttsvd_and_bound(eps):
    """Rounding is Algorithm 1 on the represented tensor: the same ranks as the
    dense TT-SVD, the same tensor, and the error within eps ||c||."""
    big = _rand_tt([1, 3, 3, 3, 1], [4, 3, 4, 3], seed=3)
    small = _rand_tt([1, 2, 4, 2, 1], [4, 3, 4, 3], seed=4, scale=0.05)
    c = _tt_sum(big, small)
    v = O.tt_full(c)
    r, tails = O.tt_round(c, eps)
    s, tails_s = O.tt_svd(v.reshape(4, 3, 4, 3, order="F"), eps)
    assert [G.shape[2] for G in r] == [G.shape[2] for G in s]
    w = O.tt_full(r)
    assert np.linalg.norm(w - O.tt_full(s)) <= 1e-10 * np.linalg.norm(v)
    err = np.linalg.norm(w - v)
    assert err <= eps * np.linalg.norm(v) * (1 + 1e-12)
    assert err <= np.sqrt(np.sum(np.square(tails))) * (1 + 1e-9) + 1e-14 * np.linalg.norm(v)


def test_round_floor_is_absolute_accuracy():
    """With a floor, the rounding accuracy is max(eps ||c||, floor): a small
    tensor rounded against a larger absolute scale keeps fewer ranks and
    stays within the floor."""
    big = _rand_tt([1, 3, 3, 3, 1], [4, 3, 4, 3], seed=13)
    small = _rand_tt([1, 2, 4, 2, 1], [4, 3, 4, 3], seed=14, scale=0.05)
    c = _tt_sum(big, small)
    c[0] = c[0] * 1e-3                                  # ||c|| is about 1e-3 of the scale below
    v = O.tt_full(c)
    scale = 1e3 * np.linalg.norm(v)
    r_rel, _ = O.tt_round(c, 1e-6)
    r_abs, _ = O.tt_round(c, 1e-6, floor=1e-3 * scale)
    assert np.linalg.norm(O.tt_full(r_abs) - v) <= 1e-3 * scale * (1 + 1e-12)
    assert sum(G.shape[2] for G in r_abs) < sum(G.shape[2] for G in r_rel)
    # a floor below eps ||c|| changes nothing
    r_low, _ = O.tt_round(c, 1e-6, floor=1e-12 * np.linalg.norm(v))
    assert [G.shape for G in r_low] == [G.shape for G in r_rel]


def test_round_two_cores_is_truncated_svd():
    """d = 2: the rounded TT is the truncated SVD of the 2-D unfolding
    (Eckart-Young), with the smallest rank whose tail is <= eps ||c||."""
    g = I.rng(5)
    U, _ = np.linalg.qr(g.standard_normal((6, 6)))
    V, _ = np.linalg.qr(g.standard_normal((7, 6)))
    sv = np.array([5.0, 2.0, 1.0, 1e-2, 1e-4, 1e-6])
    M = (U * sv) @ V.T
    c = [U.reshape(1, 6, 6) * sv, V.T.reshape(6, 7, 1)]
    full = O.tt_full(c).reshape(6, 7, order="F")
    assert np.allclose(full, M, atol=1e-13)
    eps = 1.5e-2 / np.linalg.norm(sv)        # tail of rank 3 is ~1.0e-2 < eps ||M||
    r, tails = O.tt_round(c, eps)
    assert r[0].shape[2] == 3
    best = (U[:, :3] * sv[:3]) @ V[:, :3].T
    assert np.allclose(O.tt_full(r).reshape(6, 7, order="F"), best, atol=1e-12)
    assert tails[0] == pytest.approx(np.linalg.norm(sv[3:]), rel=1e-10)


def test_round_matrix_and_orthonormal_cores():
    c = _rand_tt([1, 5, 6, 1], [4, 4, 4], seed=6)
    r, _ = O.tt_round(c, 1e-12)
    for G in r[:-1]:
        Mk = G.reshape(-1, G.shape[2], order="F")
        assert np.allclose(Mk.T @ Mk, np.eye(G.shape[2]), atol=1e-12)


def test_diric_is_dirichlet_kernel_sum():
    """diric(t, nu) = (1/nu) sum_{k=0}^{nu-1} cos((k - (nu-1)/2) t), including
    the values at t = 2 pi k."""
    g = I.rng(7)
    t = np.concatenate([g.uniform(-20, 20, 200), 2 * np.pi * np.arange(-3, 4)])
    for nu in (10, 7):
        ref = sum(np.cos((k - (nu - 1) / 2) * t) for k in range(nu)) / nu
        assert np.allclose(O.diric(t, nu), ref, atol=1e-12), nu


def test_diric_rhs_separable_in_morton_order():
    L = 3
    f = O.diric_rhs(L)
    P = O.morton_points(L)
    side = 1 << L
    grid = np.zeros((side, side, side))
    grid[P[:, 0], P[:, 1], P[:, 2]] = f
    h = 1.0 / side
    phi = O.diric(2 * np.pi * (np.arange(side) + 0.5) * h, 10)
    assert np.allclose(grid, np.einsum("i,j,k->ijk", phi, phi, phi), atol=1e-14)
    # QTT ranks over the octree digits: 8 at every interior cut at L = 3
    cores, _ = O.tt_svd(f.reshape(8, 8, 8, order="F"), 1e-12)
    assert [G.shape[2] for G in cores] == [8, 8, 1]


def test_matmul_and_lincomb_dense():
    A = I.gaussian_qtt([1, 3, 2, 1], [2, 3, 2], [3, 2, 2], seed=8)
    B = I.gaussian_qtt([1, 2, 4, 1], [3, 2, 2], [2, 2, 3], seed=9)
    C = O.qtt_matmul(A, B)
    assert [G.shape[3] for G in C] == [6, 8, 1]
    assert np.allclose(O.qtt_to_dense(C), O.qtt_to_dense(A) @ O.qtt_to_dense(B), atol=1e-13)
    A2 = I.gaussian_qtt([1, 2, 2, 1], [2, 3, 2], [3, 2, 2], seed=10)
    S = O.qtt_lincomb([(2.0, A), (-0.5, A2), (1.0, A)])
    ref = 3.0 * O.qtt_to_dense(A) - 0.5 * O.qtt_to_dense(A2)
    assert np.allclose(O.qtt_to_dense(S), ref, atol=1e-13)
    Iq = O.qtt_identity([2, 3, 2])
    assert np.array_equal(O.qtt_to_dense(Iq), np.eye(12))


@pytest.mark.parametrize("ranks,modes", [([1, 4, 1], [8, 8]), ([1, 3, 4, 3, 1], [2] * 4),
                                          ([1, 3, 4, 4, 3, 1], [2] * 5)])
def test_newton_schulz_follows_dense_iteration(ranks, modes):
    """Without truncation (eps = 1e-14) the QTT iterates are the dense
    iterates X <- X (2I - A X); the residual norm squares each step (up to the
    dense bound ||R^2||_F <= ||R||_F^2) and the limit is inv(A).  (Small N:
    the exact iterates' ranks reach the size of the unfoldings.)"""
    Ac, Aic = I.perturbed_identity_pair(ranks, modes, seed=11)
    A = O.qtt_to_dense(Ac)
    X, hist = O.newton_schulz(Ac, Aic, 1e-14, max_iter=4)
    Xd = O.qtt_to_dense(Aic)
    n = A.shape[0]
    dense_hist = []
    for t in range(len(hist)):
        R = np.eye(n) - A @ Xd
        dense_hist.append(np.linalg.norm(R) / np.sqrt(n))
        if t < len(hist) - 1:
            Xd = Xd @ (2 * np.eye(n) - A @ Xd)
    assert np.allclose(hist, dense_hist, rtol=1e-6, atol=1e-13)
    assert np.linalg.norm(O.qtt_to_dense(X) - Xd) <= 1e-12 * np.linalg.norm(Xd)
    for h0, h1 in zip(dense_hist, dense_hist[1:]):
        assert h1 <= np.sqrt(n) * h0 ** 2 * (1 + 1e-9) + 1e-14
    Ainv = np.linalg.inv(A)
    assert np.linalg.norm(Xd - Ainv) <= 1e-12 * np.linalg.norm(Ainv)


def test_newton_schulz_truncated_accuracy():
    """With rounding at eps the iteration stalls near eps: the final residual
    ||I - A X|| is within a small multiple of eps, and X is inv(A) to that
    accuracy."""
    Ac, Aic = I.perturbed_identity_pair([1, 3, 4, 4, 3, 1], [2] * 5, seed=12)
    X, hist = O.newton_schulz(Ac, Aic, 1e-8, max_iter=6)
    A = O.qtt_to_dense(Ac)
    R = np.eye(A.shape[0]) - A @ O.qtt_to_dense(X)
    assert np.linalg.norm(R) / np.sqrt(A.shape[0]) <= 1e-6
    assert hist[-1] <= 1e-6


def test_newton_schulz_adaptive_rounding():
    """theta > 0 rounds early iterates coarser (accuracy theta h_t^2): the
    same final accuracy as the plain rule, never larger ranks at the end, and
    the residual still squares until it reaches the rounding level."""
    Ac, Aic = I.perturbed_identity_pair([1, 3, 4, 4, 3, 1], [2] * 5, seed=15)
    X1, h1 = O.newton_schulz(Ac, Aic, 1e-9, max_iter=6)
    X2, h2 = O.newton_schulz(Ac, Aic, 1e-9, max_iter=6, theta=0.1)
    A = O.qtt_to_dense(Ac)
    Ainv = np.linalg.inv(A)
    for X in (X1, X2):
        assert np.linalg.norm(O.qtt_to_dense(X) - Ainv) <= 1e-7 * np.linalg.norm(Ainv)
    assert max(G.shape[3] for G in X2) <= max(G.shape[3] for G in X1)
    assert h2[-1] <= 1e-7 and h2[1] <= 2 * np.sqrt(32) * h2[0] ** 2
