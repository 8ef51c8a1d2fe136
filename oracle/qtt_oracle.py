"""Plain FP64 CPU oracle for the QTT matrix-by-full-vector product.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may call it.  It shares no code with the HIP library.

Every function is written for a reader holding the paper
(Corona, Rahimian, Zorin, "A Tensor-Train accelerated solver for integral
equations in complex geometries", arXiv:1511.06029):

* index convention -- section 2.1 (Nomenclature): multi-indices are flattened
  in Matlab order, so ``i = i_1 + m_1*(i_2 + m_2*(i_3 + ...))``; the first
  index is the fastest.  Core 1 is the finest tree level (section 2.4,
  hierarchical tensorization: levels are numbered from the finest).
* TT format -- section 2.2, Definition of the TT decomposition (eq. TTdeccores),
  with dummy ranks r_0 = r_d = 1.
* QTT matrix over the product tree -- section 3 (tensorized matrix
  A_T(b_1..b_d) with b_k = (i_k, j_k)); a core is G_k(a_{k-1}, i_k, j_k, a_k).
* matrix by full vector -- the product Algorithm 2 (section 4.2,
  alg:TT-matvec) computes, contracted here core by core from the TT formula.
* matrix by compressed vector -- section 4.2 (QTT compressed matrix-vector
  product): the cores of c = A b are the contractions over j_k of A's and
  b's cores, with the rank pairs merged (ranks multiply).
* TT-SVD -- section 2.3, Algorithm 1 (alg:TT-dec).
* non-translation-invariant operators -- section 3, the matrix form of the
  Nystrom discretisation (eq. nystrom): A = a I + B K W C with B, C, W
  diagonal (entries b(x_i), c(y_j), w_j).
* TT rounding -- the TT decomposition that Algorithm 1 (section 2.3) gives
  for a tensor that is itself handed over in TT form, computed from its
  cores (the compressed product of section 4.2 has ranks that multiply; the
  "QTT solve" of section 5.2 rounds them back).
* the right-hand side of the volume experiments -- section 5.2: f(x, y, z) =
  phi(x) phi(y) phi(z), phi(t) = diric(2 pi t, 10) (eq. diric).
* QTT inversion -- the Newton-Hotelling-Schulz iteration that section 1.3
  names among the QTT inversion methods, X <- X (2 I - A X), in QTT form
  with the matrix-matrix product (ranks multiply, as in the proof of the
  corollary on non-translation-invariant kernels in section 3) and rounding
  after each product.
* outer Krylov solver -- section 5.3 (boundary integral equations): the
  compressed approximate inverse preconditions an unrestarted GMRES with a
  relative-residual tolerance of 1e-8.  Because a low-precision inverse apply
  is linear only up to rounding, the solver here is the flexible variant
  (FGMRES, Saad 1993), which keeps the preconditioned directions.

Array conventions used throughout: a QTT matrix is a list of FP64 numpy arrays
``cores[k]`` of shape ``(r_{k-1}, m_k, n_k, r_k)``; a block of vectors is an
``(N, K)`` array whose columns are the right-hand sides.

Everything is FP64.  Reshapes that the paper writes in Matlab notation use
``order='F'`` so that they read the same way.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "qtt_shapes", "qtt_entry", "qtt_to_dense", "qtt_apply_alg2",
    "alg2_flops", "tt_svd", "qtt_matrix_from_dense", "morton_points",
    "volume_self_term", "volume_matrix", "volume_apply_direct",
    "richardson_solve", "fgmres_solve", "nti_apply", "qtt_matvec_compressed",
    "tt_full", "tt_round", "diric", "diric_rhs", "qtt_matmul", "qtt_lincomb", "qtt_identity",
    "qtt_round_matrix", "newton_schulz",
]


# --------------------------------------------------------------------------
# shapes and the plain definition
# --------------------------------------------------------------------------

def qtt_shapes(cores):
    """Return (ranks, m, n) of a QTT matrix, checking r_0 = r_d = 1 and that
    neighbouring cores agree on their shared rank (TT definition, sec. 2.2)."""
    d = len(cores)
    if d < 1:
        raise ValueError("a QTT matrix needs at least one core")
    ranks = [int(cores[0].shape[0])]
    m, n = [], []
    for k, G in enumerate(cores):
        if G.ndim != 4:
            raise ValueError(f"core {k} must be 4-D (r_prev, m, n, r_next)")
        if G.shape[0] != ranks[-1]:
            raise ValueError(f"rank mismatch entering core {k}")
        m.append(int(G.shape[1]))
        n.append(int(G.shape[2]))
        ranks.append(int(G.shape[3]))
    if ranks[0] != 1 or ranks[-1] != 1:
        raise ValueError("boundary ranks r_0 and r_d must be 1")
    return ranks, m, n


def _digits(index, modes):
    """Split a flat index into digits, first digit fastest (sec. 2.1)."""
    out = []
    for size in modes:
        out.append(index % size)
        index //= size
    return out


def qtt_entry(cores, i, j):
    """One matrix entry A(i, j) straight from the TT definition (eq. TTdeccores
    applied to the product-tree tensor of sec. 3): the product of the
    r_{k-1} x r_k matrices G_k(:, i_k, j_k, :) over k, a 1 x 1 result."""
    _, m, n = qtt_shapes(cores)
    idig = _digits(int(i), m)
    jdig = _digits(int(j), n)
    v = np.ones((1, 1))
    for G, ik, jk in zip(cores, idig, jdig):
        v = v @ G[:, ik, jk, :]
    return float(v[0, 0])


def qtt_to_dense(cores):
    """Dense M x N matrix represented by the cores (sec. 3, tensorized matrix
    A_T(b_1, ..., b_d) = A(overline{i_1..i_d}, overline{j_1..j_d})).

    The chain of cores is contracted over the rank indices, giving an array
    with axes (i_1, j_1, i_2, j_2, ..., i_d, j_d); the i axes and j axes are
    then flattened with the first digit fastest."""
    _, m, n = qtt_shapes(cores)
    d = len(cores)
    T = cores[0]
    for G in cores[1:]:
        T = np.tensordot(T, G, axes=([T.ndim - 1], [0]))
    T = T.reshape(T.shape[1:-1])                      # (m1, n1, ..., md, nd)
    perm = [2 * k for k in range(d)] + [2 * k + 1 for k in range(d)]
    T = T.transpose(perm)                             # (m1..md, n1..nd)
    return T.reshape(int(np.prod(m)), int(np.prod(n)), order="F")


# --------------------------------------------------------------------------
# the matrix by full-vector product (computed by Alg. 2 in section 4.2)
# --------------------------------------------------------------------------

def _contract_digits(cores, x):
    """y = A x for one vector, contracting the digit tensor of x with the cores.

    Written from the TT entry formula: with x viewed as the tensor
    x[j_1, ..., j_d] (first digit fastest),

        y[i_1..i_d] = sum over j_1..j_d and the rank indices of
                      G_1[1, i_1, j_1, a_1] G_2[a_1, i_2, j_2, a_2] ... G_d[a_{d-1}, i_d, j_d, 1]
                      x[j_1, ..., j_d].

    The sums are taken one core at a time, finest level first.  After core k
    the partial result is a tensor W_k[a_k, j_{k+1}, ..., j_d, i_1, ..., i_k]:
    the source digits j_1..j_k are summed out, the target digits i_1..i_k are
    free, and a_k links it to the cores still to come.  This is the order in
    which Alg. 2 visits the cores; here it is a plain tensor contraction with
    no blocking or layout of its own."""
    W = np.asarray(x, dtype=np.float64).reshape([G.shape[2] for G in cores], order="F")
    W = W[np.newaxis]                                  # W_0[a_0 = 0, j_1, ..., j_d]
    for G in cores:
        # W_k[i_k, a_k, rest] = sum_{a_{k-1}, j_k} G_k[a_{k-1}, i_k, j_k, a_k] W_{k-1}[a_{k-1}, j_k, rest]
        T = np.tensordot(G, W, axes=([0, 2], [0, 1]))
        W = np.moveaxis(T, 0, -1)                      # i_k joins the target digits, slowest
    # W_d[a_d = 0, i_1, ..., i_d]; flatten the target digits first-fastest
    return W[0].reshape(-1, order="F")


def qtt_apply_alg2(cores, X):
    """Y = A X for a block of vectors: the product that Alg. 2 (section 4.2)
    computes, taken column by column by _contract_digits.

    X: (N,) or (N, K) FP64.  Returns an array of shape (M,) or (M, K)."""
    _, m, n = qtt_shapes(cores)
    X = np.asarray(X, dtype=np.float64)
    N = int(np.prod(n))
    if X.shape[0] != N:
        raise ValueError(f"X has {X.shape[0]} rows, the operator has {N} columns")
    if X.ndim == 1:
        return _contract_digits(cores, X)
    Y = np.empty((int(np.prod(m)), X.shape[1]))
    for c in range(X.shape[1]):
        Y[:, c] = _contract_digits(cores, X[:, c])
    return Y


def qtt_matvec_compressed(A_cores, b_cores):
    """Cores of c = A b when b is itself in TT form (section 4.2, compressed
    matrix-vector product):

        G^c_k(alpha + rA_{k-1} beta, i, alpha' + rA_k beta')
            = sum_j G^A_k(alpha, i, j, alpha') G^b_k(beta, j, beta')

    The merged rank index puts the matrix's rank first (fastest), the
    paper's merged-index order.  b_cores[k] has shape (rb_{k-1}, n_k, rb_k);
    the result has shape (rA_{k-1} rb_{k-1}, m_k, rA_k rb_k)."""
    out = []
    for GA, Gb in zip(A_cores, b_cores):
        ra0, m, n, ra1 = GA.shape
        rb0, n2, rb1 = Gb.shape
        if n2 != n:
            raise ValueError("mode sizes of A and b differ")
        T = np.einsum("aijc,bjd->baidc", GA, Gb)   # [beta, alpha, i, beta', alpha']
        out.append(T.reshape(rb0 * ra0, m, rb1 * ra1))
    return out


def alg2_flops(ranks, m, n):
    """Floating-point operations of one Algorithm-2 sweep for one vector.

    Core k multiplies an (r_k m_k) x (r_{k-1} n_k) matrix by a matrix with
    C_k = prod_{l<k} m_l * prod_{l>k} n_l columns: 2 * r_k m_k r_{k-1} n_k C_k
    flops.  For square modes this is 2 m_k r_{k-1} r_k N, the count given after
    Algorithm 2 once its rank subscripts are read as those of M_k's size."""
    d = len(m)
    total = 0
    for k in range(d):
        cols = int(np.prod(m[:k], dtype=np.int64) * np.prod(n[k + 1:], dtype=np.int64))
        total += 2 * ranks[k + 1] * m[k] * ranks[k] * n[k] * cols
    return int(total)


# --------------------------------------------------------------------------
# Algorithm 1: TT-SVD, and the QTT matrix of a dense matrix
# --------------------------------------------------------------------------

def _keep_rank(s, delta):
    """Smallest r >= 1 whose discarded singular values s_r, s_{r+1}, ... have
    a Euclidean norm of at most delta (the optimal rank-r error of the
    unfolding, Eckart-Young), and that norm."""
    tail = np.sqrt(np.cumsum((s ** 2)[::-1])[::-1])     # tail[r] = ||s[r:]||
    tail = np.append(tail, 0.0)
    r = 1
    while r < len(s) and tail[r] > delta:
        r += 1
    return r, float(tail[r])


def tt_svd(tensor, eps):
    """TT decomposition of a dense tensor by successive truncated SVDs of its
    unfoldings (Alg. 1, section 2.3, with the truncated SVD as the low-rank
    routine and the per-unfolding accuracy eps ||A||_F / sqrt(d-1)).

    The modes are split off one at a time from the front.  The remainder R is
    kept as a tensor R[a_{k-1}, i_k, i_{k+1}, ..., i_d]; its k-th unfolding
    groups (a_{k-1}, i_k) into rows.  The left singular vectors of that
    unfolding, cut to the rank _keep_rank allows, are core k; the singular
    values times the right singular vectors become the next remainder, with
    the new rank index in front.  The last remainder is core d.

    Returns (cores, tails): cores[k] has shape (r_{k-1}, n_k, r_k), and
    tails[k] is the Frobenius norm cut away from unfolding k+1."""
    A = np.asarray(tensor, dtype=np.float64)
    modes = A.shape
    d = len(modes)
    if d == 1:
        return [A.reshape(1, modes[0], 1).copy()], []
    delta = eps * np.linalg.norm(A) / np.sqrt(d - 1)
    R = A[np.newaxis]                                   # R[a_0 = 0, i_1, ..., i_d]
    cores, tails = [], []
    for k in range(d - 1):
        ra, nk = R.shape[0], R.shape[1]
        rest = R.shape[2:]
        U, s, Vt = np.linalg.svd(R.reshape(ra * nk, -1, order="F"), full_matrices=False)
        r, cut = _keep_rank(s, delta)
        tails.append(cut)
        cores.append(U[:, :r].reshape(ra, nk, r, order="F"))
        R = (s[:r, None] * Vt[:r]).reshape((r,) + rest, order="F")
    cores.append(R.reshape(R.shape[0], modes[-1], 1, order="F"))
    return cores, tails


def qtt_matrix_from_dense(A, m, n, eps):
    """QTT matrix of a dense M x N matrix (sec. 3 tensorization + Algorithm 1).

    The matrix is viewed as the d-dimensional tensor over the product tree,
    A_T(b_1..b_d) with b_k = overline{i_k j_k} (i_k fastest), then compressed.
    Returns (cores, tails) with cores[k] of shape (r_{k-1}, m_k, n_k, r_k)."""
    d = len(m)
    A = np.asarray(A, dtype=np.float64)
    T = A.reshape(tuple(m) + tuple(n), order="F")     # axes (i_1..i_d, j_1..j_d)
    perm = []
    for k in range(d):
        perm += [k, d + k]
    T = T.transpose(perm)                             # (i_1, j_1, ..., i_d, j_d)
    T = T.reshape(tuple(m[k] * n[k] for k in range(d)), order="F")
    tt, tails = tt_svd(T, eps)
    cores = [G.reshape(G.shape[0], m[k], n[k], G.shape[2], order="F")
             for k, G in enumerate(tt)]
    return cores, tails


# --------------------------------------------------------------------------
# the volume operator of the numerical experiments (sec. 5.2)
# --------------------------------------------------------------------------

def morton_points(L):
    """Integer cell coordinates (ix, iy, iz) of a (2^L)^3 grid listed in
    octree (Morton) order: point index i = sum_k i_k 8^{k-1}, where the level-k
    octant digit is i_k = 4 z_bit + 2 y_bit + x_bit of bit k-1 of each
    coordinate (level 1 = finest, sec. 2.4; ordering of sec. 5.2)."""
    side = 1 << L
    N = side ** 3
    idx = np.arange(N, dtype=np.int64)
    ix = np.zeros(N, dtype=np.int64)
    iy = np.zeros(N, dtype=np.int64)
    iz = np.zeros(N, dtype=np.int64)
    for k in range(L):
        digit = (idx >> (3 * k)) & 7
        ix |= (digit & 1) << k
        iy |= ((digit >> 1) & 1) << k
        iz |= ((digit >> 2) & 1) << k
    return np.stack([ix, iy, iz], axis=1)


def volume_self_term(h, sub=8):
    """Diagonal self term: midpoint rule with sub^3 sub-cells for the integral
    of 1/(4 pi |x - y|) over the cell centred at x (no sub-cell midpoint hits
    the singularity).  Used in place of the punctured trapezoid of sec. 5.2."""
    t = (np.arange(sub) + 0.5) / sub - 0.5
    u = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
    return float(np.sum((h / sub) ** 3 / (4.0 * np.pi * h * np.linalg.norm(u, axis=1))))


def volume_matrix(L):
    """Nystrom matrix A = I + K W (eq. nystrom with a = 1, b = c = 1, w = h^3)
    of the Laplace single-layer kernel 1/(4 pi r) on the cell centres of a
    (2^L)^3 grid on [0,1]^3 in Morton order; diagonal 1 + self term."""
    side = 1 << L
    h = 1.0 / side
    P = (morton_points(L) + 0.5) * h
    diff = P[:, None, :] - P[None, :, :]
    dist = np.sqrt(np.sum(diff * diff, axis=-1))
    np.fill_diagonal(dist, 1.0)
    A = h ** 3 / (4.0 * np.pi * dist)
    np.fill_diagonal(A, 1.0 + volume_self_term(h))
    return A


def volume_apply_direct(L, X):
    """y = A x for the volume operator by direct summation over grid
    coordinates, y_i = (1 + s) x_i + sum_{j != i} h^3 / (4 pi |p_i - p_j|) x_j,
    evaluated in natural (x fastest) grid order as a zero-padded 3-D
    convolution with scipy's FFT, then listed in Morton order.  It never forms
    the matrix and never uses the octree digits except to reorder."""
    from scipy.signal import fftconvolve
    side = 1 << L
    h = 1.0 / side
    s = volume_self_term(h)
    off = np.arange(-(side - 1), side)
    dz, dy, dx = np.meshgrid(off, off, off, indexing="ij")
    r = h * np.sqrt(dx * dx + dy * dy + dz * dz)
    r[side - 1, side - 1, side - 1] = 1.0
    kern = h ** 3 / (4.0 * np.pi * r)
    kern[side - 1, side - 1, side - 1] = 0.0
    pts = morton_points(L)
    X = np.asarray(X, dtype=np.float64)
    one = X.ndim == 1
    X2 = X[:, None] if one else X
    Y = np.empty_like(X2)
    for c in range(X2.shape[1]):
        grid = np.zeros((side, side, side))
        grid[pts[:, 2], pts[:, 1], pts[:, 0]] = X2[:, c]
        conv = fftconvolve(grid, kern, mode="full")
        conv = conv[side - 1:2 * side - 1, side - 1:2 * side - 1, side - 1:2 * side - 1]
        Y[:, c] = conv[pts[:, 2], pts[:, 1], pts[:, 0]] + (1.0 + s) * X2[:, c]
    return Y[:, 0] if one else Y


# --------------------------------------------------------------------------
# non-translation-invariant operators (sec. 3, eq. nystrom)
# --------------------------------------------------------------------------

def nti_apply(K_cores, a, b, wc, X):
    """Y = (a I + B K W C) X with K a QTT matrix and B = diag(b), W C =
    diag(wc) (the Nystrom matrix of section 3, eq. nystrom; wc holds the
    products w_j c(y_j)).  b or wc = None stands for all ones.  Written as
    the definition reads: scale the input, apply K by Algorithm 2, scale the
    output, add a X."""
    X = np.asarray(X, dtype=np.float64)
    one = X.ndim == 1
    X2 = X[:, None] if one else X
    Xs = X2 if wc is None else np.asarray(wc, dtype=np.float64)[:, None] * X2
    T = qtt_apply_alg2(K_cores, Xs)
    if b is not None:
        T = np.asarray(b, dtype=np.float64)[:, None] * T
    Y = T + a * X2 if a != 0.0 else T
    return Y[:, 0] if one else Y


# --------------------------------------------------------------------------
# the solve: direct inverse apply plus iterative refinement
# --------------------------------------------------------------------------

def richardson_solve(A_cores, Ainv_cores, F, rtol=1e-8, max_iter=50):
    """sigma with A sigma = F by refinement with the compressed inverse:
    x = 0, r = F; repeat { x += Ainv r ; r = F - A x } until
    ||r_c|| <= rtol ||F_c|| for every column c.  The first pass is the paper's
    direct solve sigma = Ainv f (sec. 5); the later passes correct it.

    Returns (X, history) where history[t] holds the per-column relative
    residuals after pass t+1."""
    F = np.asarray(F, dtype=np.float64)
    one = F.ndim == 1
    F2 = F[:, None] if one else F
    fn = np.linalg.norm(F2, axis=0)
    fn[fn == 0] = 1.0
    X = np.zeros_like(F2)
    R = F2.copy()
    history = []
    for _ in range(max_iter):
        X = X + qtt_apply_alg2(Ainv_cores, R)
        R = F2 - qtt_apply_alg2(A_cores, X)
        rel = np.linalg.norm(R, axis=0) / fn
        history.append(rel)
        if np.all(rel <= rtol):
            break
    return (X[:, 0] if one else X), history


# --------------------------------------------------------------------------
# the outer Krylov solver: flexible GMRES, right preconditioner (sec. 5.3)
# --------------------------------------------------------------------------

def fgmres_solve(apply_A, apply_M, F, rtol=1e-8, max_iter=50):
    """sigma with A sigma = F by unrestarted flexible GMRES, one column at a
    time, as section 5.3 uses GMRES (no restart, relative-residual tolerance)
    with the compressed inverse as right preconditioner.

    The steps are Saad's FGMRES (SIAM J. Sci. Comput. 14, 1993), written out
    plainly: x_0 = 0, v_1 = f / ||f||; for j = 1, 2, ...
        z_j = M v_j;  w = A z_j;
        modified Gram-Schmidt: h_ij = <w, v_i>, w -= h_ij v_i  (i = 1..j);
        h_{j+1,j} = ||w||;  v_{j+1} = w / h_{j+1,j};
        Givens rotations reduce the (j+1) x j Hessenberg matrix to upper
        triangular form; the last rotated right-hand-side entry |g_{j+1}| is
        the residual norm ||f - A x_j||;
    stop when |g_{j+1}| <= rtol ||f|| (or on breakdown h_{j+1,j} = 0); then
    x = Z y with R y = g (the stored z_j, not M applied to V y, so M may change
    from one step to the next).

    apply_A, apply_M: functions of one FP64 vector (N,) returning (N,);
    apply_M = None means no preconditioner (z_j = v_j).
    Returns (X, history, iters): history[c][t] = |g_{t+2}| / ||f_c|| after step
    t+1 of column c, iters[c] = the steps that column took."""
    F = np.asarray(F, dtype=np.float64)
    one = F.ndim == 1
    F2 = F[:, None] if one else F
    N, K = F2.shape
    X = np.zeros_like(F2)
    history, iters = [], []
    for c in range(K):
        f = F2[:, c]
        beta = float(np.linalg.norm(f))
        hist = []
        if beta == 0.0:
            history.append(hist)
            iters.append(0)
            continue
        V = [f / beta]
        Z = []
        H = np.zeros((max_iter + 1, max_iter))
        g = np.zeros(max_iter + 1)
        g[0] = beta
        cs = np.zeros(max_iter)
        sn = np.zeros(max_iter)
        k = 0
        for j in range(max_iter):
            z = V[j] if apply_M is None else np.asarray(apply_M(V[j]), dtype=np.float64)
            Z.append(z)
            w = np.asarray(apply_A(z), dtype=np.float64).copy()
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            hnext = float(np.linalg.norm(w))
            H[j + 1, j] = hnext
            for i in range(j):
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -sn[i] * a + cs[i] * b
            d = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            hist.append(abs(g[j + 1]) / beta)
            k = j + 1
            if abs(g[j + 1]) <= rtol * beta or hnext == 0.0:
                break
            V.append(w / hnext)
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        X[:, c] = sum(y[i] * Z[i] for i in range(k))
        history.append(hist)
        iters.append(k)
    return (X[:, 0] if one else X), history, iters


# --------------------------------------------------------------------------
# TT vectors: expansion and rounding
# --------------------------------------------------------------------------

def tt_full(cores):
    """The vector a TT decomposition with cores[k] of shape (r_{k-1}, n_k, r_k)
    represents (eq. TTdeccores), flattened first index fastest (section 2.1)."""
    T = np.ones((1, 1))
    for G in cores:
        T = np.tensordot(T, G, axes=([T.ndim - 1], [0]))
    return T.reshape(-1, order="F")  # axes (a_0, i_1, ..., i_d, a_d), a_0 = a_d = 0


def tt_round(cores, eps, floor=0.0):
    """The TT decomposition that Algorithm 1 (truncated SVDs, per-unfolding
    accuracy eps ||c||_F / sqrt(d-1)) computes for the tensor c that `cores`
    represent, without expanding c.

    Why it can be done core by core: if cores k+1..d are right-orthonormal
    (each core, as the r_{k-1} x (n_k r_k) matrix of its entries, has
    orthonormal rows), the k-th unfolding of c is (its first k cores,
    contracted) times a matrix with orthonormal rows, so it has the singular
    values and left singular vectors of the first factor.  Hence:
      1. right to left, k = d..2: QR of core k's transposed matrix,
         core k <- Q^T (orthonormal rows), core k-1 <- core k-1 R^T;
      2. left to right, k = 1..d-1: SVD of core k as the (r_{k-1} n_k) x r_k
         matrix, keep the rank _keep_rank allows (tail <= eps ||c|| /
         sqrt(d-1)), core k <- U, core k+1 <- (S V^T) core k+1.
    floor > 0 replaces eps ||c|| by max(eps ||c||, floor): an absolute
    accuracy for a tensor whose own norm is not the scale that matters.
    Returns (cores, tails) as tt_svd does."""
    G = [np.array(c, dtype=np.float64, copy=True) for c in cores]
    d = len(G)
    for k in range(d - 1, 0, -1):
        r0, n, r1 = G[k].shape
        q, rr = np.linalg.qr(G[k].reshape(r0, n * r1, order="F").T)      # (n r1) x r', r' x r0
        G[k] = q.T.reshape(q.shape[1], n, r1, order="F")
        G[k - 1] = np.tensordot(G[k - 1], rr.T, axes=([2], [0]))        # r_{k-2} x n x r'
    norm = float(np.linalg.norm(G[0]))
    if d == 1:
        return G, []
    delta = max(eps * norm, floor) / np.sqrt(d - 1)
    tails = []
    for k in range(d - 1):
        r0, n, r1 = G[k].shape
        U, sv, Vt = np.linalg.svd(G[k].reshape(r0 * n, r1, order="F"), full_matrices=False)
        r, cut = _keep_rank(sv, delta)
        tails.append(cut)
        G[k] = U[:, :r].reshape(r0, n, r, order="F")
        G[k + 1] = np.tensordot(sv[:r, None] * Vt[:r], G[k + 1], axes=([1], [0]))
    return G, tails


# --------------------------------------------------------------------------
# the right-hand side of the volume experiments (section 5.2)
# --------------------------------------------------------------------------

def diric(t, nu):
    """The periodic sinc function of eq. diric: sin(nu t / 2) / (nu sin(t / 2)),
    and (-1)^(k (nu - 1)) at t = 2 pi k."""
    t = np.asarray(t, dtype=np.float64)
    k = np.round(t / (2.0 * np.pi))
    at_pole = np.isclose(t, 2.0 * np.pi * k, rtol=0.0, atol=1e-12)
    den = nu * np.sin(t / 2.0)
    safe = np.where(at_pole, 1.0, den)
    val = np.sin(nu * t / 2.0) / safe
    return np.where(at_pole, (-1.0) ** (k * (nu - 1)), val)


def diric_rhs(L, nu=10):
    """f(x, y, z) = phi(x) phi(y) phi(z), phi(t) = diric(2 pi t, nu), at the
    cell centres of the (2^L)^3 grid on [0,1]^3, listed in Morton order
    (section 5.2's right-hand side, on the grid of volume_matrix)."""
    h = 1.0 / (1 << L)
    P = (morton_points(L) + 0.5) * h
    phi = diric(2.0 * np.pi * P, nu)
    return phi[:, 0] * phi[:, 1] * phi[:, 2]


# --------------------------------------------------------------------------
# QTT matrices: product, linear combination, rounding, Newton-Schulz
# --------------------------------------------------------------------------

def qtt_identity(m):
    """Rank-1 QTT of the identity: cores delta(i_k, j_k)."""
    return [np.eye(mk).reshape(1, mk, mk, 1) for mk in m]


def qtt_matmul(A_cores, B_cores):
    """Cores of the product A B: C_k(alpha + rA beta, i, j, alpha' + rA beta') =
    sum_l A_k(alpha, i, l, alpha') B_k(beta, l, j, beta').  The ranks multiply
    (the merged rank index puts A's rank first, as qtt_matvec_compressed)."""
    out = []
    for GA, GB in zip(A_cores, B_cores):
        ra0, m, l, ra1 = GA.shape
        rb0, l2, n, rb1 = GB.shape
        if l2 != l:
            raise ValueError("inner mode sizes differ")
        T = np.einsum("ailc,bljd->baijdc", GA, GB)     # [beta, alpha, i, j, beta', alpha']
        out.append(T.reshape(rb0 * ra0, m, n, rb1 * ra1))
    return out


def qtt_lincomb(terms):
    """Cores of sum_t c_t A_t for a list of (c_t, cores_t) with equal modes:
    block-diagonal interior cores, the first core a row of blocks and the last
    a column (the TT sum; ranks add).  The coefficients scale the first core."""
    d = len(terms[0][1])
    out = []
    for k in range(d):
        blocks = [(c if k == 0 else 1.0) * cores[k] for c, cores in terms]
        m, n = blocks[0].shape[1], blocks[0].shape[2]
        r0 = 1 if k == 0 else sum(b.shape[0] for b in blocks)
        r1 = 1 if k == d - 1 else sum(b.shape[3] for b in blocks)
        G = np.zeros((r0, m, n, r1))
        a = b = 0
        for blk in blocks:
            p, q = blk.shape[0], blk.shape[3]
            ia = slice(0, 1) if k == 0 else slice(a, a + p)
            ib = slice(0, 1) if k == d - 1 else slice(b, b + q)
            G[ia, :, :, ib] += blk
            a += p
            b += q
        out.append(G)
    return out


def qtt_round_matrix(cores, eps, floor=0.0):
    """tt_round of a QTT matrix, its cores read as TT cores of mode m_k n_k
    (row digit fastest, the index b_k = i_k + m_k j_k of section 3)."""
    shapes = [(G.shape[1], G.shape[2]) for G in cores]
    tt = [G.reshape(G.shape[0], G.shape[1] * G.shape[2], G.shape[3], order="F") for G in cores]
    out, tails = tt_round(tt, eps, floor)
    return [G.reshape(G.shape[0], m, n, G.shape[2], order="F") for G, (m, n) in zip(out, shapes)], tails


def newton_schulz(A_cores, X0_cores, eps, max_iter=20, tol=0.0, theta=0.0):
    """Approximate inverse of A by the Newton-Hotelling-Schulz iteration
    X_{t+1} = X_t (2 I - A X_t) in QTT form: each product by qtt_matmul,
    the sum by qtt_lincomb, and tt rounding (relative accuracy eps) after
    each product and after the sum.  The residual R = I - A X is rounded to
    accuracy eps ||I||_F (the scale X's accuracy is measured on), not eps
    ||R||: once X is good, R is mostly the rounding noise of the previous
    steps, whose rank relative to its own norm is not bounded.  In exact
    arithmetic I - A X_{t+1} = (I - A X_t)^2, so the iteration converges
    quadratically once ||I - A X_0|| < 1.

    theta > 0 rounds the next iterate (and 2 I - A X) to the accuracy
    max(eps, theta h_t^2) instead of eps, h_t = ||R_t||_F / ||I||_F: the
    next iterate is within about h_t^2 of the inverse, so more accuracy buys
    only rank (an early iterate has high ranks at a tight eps that the
    inverse itself does not need).

    Stops after max_iter steps or once the rounded residual matrix
    R = I - A X has ||R||_F <= tol ||I||_F.  Returns (X_cores, history) with
    history[t] = ||I - A X_t||_F / ||I||_F for t = 0, 1, ... (computed from the
    rounded QTT of A X_t, before X_{t+1} is formed)."""
    m = [G.shape[1] for G in A_cores]
    I = qtt_identity(m)
    ident_norm = float(np.sqrt(np.prod(m)))
    X = [np.array(G, dtype=np.float64) for G in X0_cores]
    history = []
    for t in range(max_iter + 1):
        AX, _ = qtt_round_matrix(qtt_matmul(A_cores, X), eps)
        R, _ = qtt_round_matrix(qtt_lincomb([(1.0, I), (-1.0, AX)]), eps, floor=eps * ident_norm)
        history.append(float(np.linalg.norm(tt_full([G.reshape(G.shape[0], -1, G.shape[3], order="F")
                                                      for G in R])) / ident_norm))
        if history[-1] <= tol or t == max_iter:
            break
        tau = max(eps, theta * history[-1] ** 2)
        Z, _ = qtt_round_matrix(qtt_lincomb([(1.0, I), (1.0, R)]), tau)      # 2 I - A X = I + R
        X, _ = qtt_round_matrix(qtt_matmul(X, Z), tau)
    return X, history
