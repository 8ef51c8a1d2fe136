"""Structured QTT matrices whose action is known without the oracle.

Test-only constructions used to pin the oracle (and, through it, the HIP
path).  Each one follows a fact stated in the paper or a textbook identity;
none of them calls the oracle's apply.
"""
from __future__ import annotations

import numpy as np


def kron_cores(mats):
    """Rank-1 QTT with G_k(0, i, j, 0) = mats[k][i, j].  By the TT definition
    A(i, j) = prod_k mats[k][i_k, j_k] with i_1 fastest, so
    A = mats[d-1] (x) ... (x) mats[0]."""
    return [np.asarray(Mk, dtype=np.float64).reshape(1, *Mk.shape, 1).copy() for Mk in mats]


def modewise_apply(mats, X):
    """(mats[d-1] (x) ... (x) mats[0]) X by contracting one mode at a time on
    the d-way view of X (first digit fastest); never forms the Kronecker
    product and never uses Algorithm 2."""
    n = [Mk.shape[1] for Mk in mats]
    m = [Mk.shape[0] for Mk in mats]
    X = np.asarray(X, dtype=np.float64)
    K = X.shape[1]
    T = X.reshape(tuple(n) + (K,), order="F")
    for k, Mk in enumerate(mats):
        T = np.tensordot(Mk, T, axes=([1], [k]))       # new axis 0 = i_k
        T = np.moveaxis(T, 0, k)
    return T.reshape(int(np.prod(m)), K, order="F")


def block_sum_cores(terms):
    """Exact QTT of sum_t (x)_k terms[t][k] with rank R = len(terms): first
    core is a row [A_1^(t)]_t, interior cores are block diagonal, last core is
    a column (TT definition, the sum of R rank-1 terms)."""
    R = len(terms)
    d = len(terms[0])
    cores = []
    for k in range(d):
        m, n = terms[0][k].shape
        r0 = 1 if k == 0 else R
        r1 = 1 if k == d - 1 else R
        G = np.zeros((r0, m, n, r1))
        for t in range(R):
            a = 0 if k == 0 else t
            b = 0 if k == d - 1 else t
            G[a, :, :, b] = terms[t][k]
        cores.append(G)
    return cores


def random_orthogonal(r, g):
    Q, R = np.linalg.qr(g.standard_normal((r, r)))
    return Q * np.sign(np.diag(R))


def gauge(cores, g):
    """G_k <- Q_{k-1}^T G_k Q_k with random orthogonal Q_k (Q_0 = Q_d = 1):
    the represented matrix is unchanged while the cores become dense."""
    d = len(cores)
    Qs = [np.ones((1, 1))]
    for k in range(d - 1):
        Qs.append(random_orthogonal(cores[k].shape[3], g))
    Qs.append(np.ones((1, 1)))
    out = []
    for k, G in enumerate(cores):
        H = np.einsum("ab,bijc->aijc", Qs[k].T, G)
        H = np.einsum("aijc,cd->aijd", H, Qs[k + 1])
        out.append(H)
    return out


def vector_tt_full(vcores):
    """Full vector from TT cores V_k(a, i_k, b) (TT definition; i_1 fastest)."""
    T = vcores[0]
    for V in vcores[1:]:
        T = np.tensordot(T, V, axes=([T.ndim - 1], [0]))
    T = T.reshape(T.shape[1:-1])
    return T.reshape(-1, order="F")


def diag_cores(vcores):
    """QTT of diag(b) from the TT of b: G^B(a, i, j, b) = delta_ij G^b(a, i, b)
    (proof of the corollary on non-translation-invariant kernels)."""
    out = []
    for V in vcores:
        r0, n, r1 = V.shape
        G = np.zeros((r0, n, n, r1))
        for i in range(n):
            G[:, i, i, :] = V[:, i, :]
        out.append(G)
    return out


def product_cores(Acores, Bcores):
    """Cores of C = A B: C_k((a, b), i, j, (a', b')) = sum_l A_k(a, i, l, a')
    B_k(b, l, j, b'); the rank indices are merged, so ranks multiply
    (matrix-matrix analogue of the compressed product, sec. 4.2)."""
    out = []
    for A, B in zip(Acores, Bcores):
        ra0, m, l, ra1 = A.shape
        rb0, l2, n, rb1 = B.shape
        assert l == l2
        C = np.einsum("aixc,bxjd->abijcd", A, B)
        out.append(C.reshape(ra0 * rb0, m, n, ra1 * rb1))
    return out


def sum_cores(Acores, Bcores):
    """Cores of A + B (TT definition: the sum of two TT products): the first
    cores side by side, the last stacked, the interior block diagonal, so the
    ranks add."""
    d = len(Acores)
    out = []
    for k, (A, B) in enumerate(zip(Acores, Bcores)):
        ra0, m, n, ra1 = A.shape
        rb0, _, _, rb1 = B.shape
        if d == 1:
            out.append(A + B)
        elif k == 0:
            out.append(np.concatenate([A, B], axis=3))
        elif k == d - 1:
            out.append(np.concatenate([A, B], axis=0))
        else:
            G = np.zeros((ra0 + rb0, m, n, ra1 + rb1))
            G[:ra0, :, :, :ra1] = A
            G[ra0:, :, :, ra1:] = B
            out.append(G)
    return out
