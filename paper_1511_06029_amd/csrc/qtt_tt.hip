// libqtt: operations on tensors in TT form -- rounding (the decomposition
// Algorithm 1 of section 2.3 gives for a tensor handed over as TT cores),
// compression of a full vector, and QTT matrix inversion by the
// Newton-Hotelling-Schulz iteration named in section 1.3.
//
// Rounding runs in two stages on the device:
//   1. Randomized range finding, right to left then left to right ("randomize
//      then orthogonalize", Al Daas, Ballard, Cazeaux, Hallman, Miedlar,
//      Pasha, Reid and Saibaba, SIAM J. Sci. Comput. 45, 2023): with Gaussian
//      sketch cores Omega_k of ranks l_k, the partial contractions
//      W_{k-1} = P_k x_3 W_k x_{2,3} Omega_k of the input with the sketch give,
//      left to right, Z = Y_k W_k, whose thin Q becomes core k, and
//      Y_{k+1} = (Q^T Y_k) P_{k+1}.  The result is left-orthonormal with
//      ranks l_k and equals the input projected onto the sketched subspaces.
//   2. Truncation to the tolerance, right to left: each core as the
//      l_{k-1} x (n_k r_k) matrix B = U diag(s) W^T (thin QR of B^T, then a
//      one-sided Jacobi SVD of the small triangular factor), the rank kept
//      by the rule of Algorithm 1 (smallest r whose discarded tail of
//      singular values is <= eps ||c|| / sqrt(d - 1)),
//      core k <- diag(1/s) U_r^T B, core k-1 <- core k-1 U_r diag(s).
// When a kept rank comes close to its sketch rank (so the sketch may have
// missed part of the range) the sketch rank is doubled, up to max_rank.
// Every product is an FP64 GEMM (gemm_kernel); the QR factorizations are
// tall-skinny Householder QRs over row blocks held in LDS (qr_block_lds_kernel,
// qr_combine_kernel; one workgroup through global memory, qr_thin_kernel,
// where the blocks do not fit), the SVDs one per workgroup
// (jacobi_svd_kernel).  The stream is
// synchronised once per core of stage 2 (the kept rank is chosen on the host).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "qtt.h"
#include "qtt_internal.hpp"
#include "qtt_tt_kernels.hpp"

using namespace qtt;

namespace {

// Device buffer of doubles owned by the host code (freed after the stream's
// work is done: every entry point synchronises before returning).
struct DBuf {
  double* p = nullptr;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p) { o.p = nullptr; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      reset();
      p = o.p;
      o.p = nullptr;
    }
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
  }
};

qtt_status_t dalloc(DBuf& b, int64_t count) {
  b.reset();
  void* ptr = nullptr;
  const size_t bytes = (size_t)std::max<int64_t>(count, 1) * 8;
  if (hipMalloc(&ptr, bytes) != hipSuccess) return fail(QTT_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed", bytes);
  b.p = static_cast<double*>(ptr);
  return QTT_OK;
}

// A TT tensor on the device: cores [r_k][n_k][r_{k+1}] row-major.
struct DevTT {
  int d = 0;
  std::vector<int64_t> n, r;
  std::vector<DBuf> core;
  int64_t len(int k) const { return r[k] * n[k] * r[k + 1]; }
};

// Cores not owned (caller's device pointers or another DevTT's).
struct TTView {
  int d = 0;
  std::vector<int64_t> n, r;
  std::vector<const double*> core;
};

TTView view(const DevTT& t) {
  TTView v;
  v.d = t.d;
  v.n = t.n;
  v.r = t.r;
  for (auto& c : t.core) v.core.push_back(c.p);
  return v;
}

unsigned grid_for(int64_t work, int64_t per_block = 256) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + per_block - 1) / per_block, 65535));
}

#define QTT_CHECK(expr)                 \
  do {                                  \
    qtt_status_t s_ = (expr);           \
    if (s_ != QTT_OK) return s_;        \
  } while (0)

const void* gemm_fn(bool ta, bool tb) {
  return ta ? (tb ? reinterpret_cast<const void*>(&gemm_kernel<true, true>)
                  : reinterpret_cast<const void*>(&gemm_kernel<true, false>))
            : (tb ? reinterpret_cast<const void*>(&gemm_kernel<false, true>)
                  : reinterpret_cast<const void*>(&gemm_kernel<false, false>));
}

// C = alpha op(A) op(B) + beta C (see gemm_kernel).  Products with few output
// tiles and a long contraction are split over the contraction (partial
// products in scratch, then summed in split order) so that they fill the GPU.
qtt_status_t gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                  const double* B, int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return QTT_OK;
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.A = A;
  g.B = B;
  g.C = C;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.alpha = alpha;
  g.beta = beta;
  g.tiles_n = (N + kGemmT - 1) / kGemmT;
  const int64_t tiles = ((M + kGemmT - 1) / kGemmT) * g.tiles_n;
  if (tiles > INT32_MAX) return fail(QTT_ERR_SHAPE, "product of %lld x %lld too large", (long long)M, (long long)N);
  int64_t splits = 1;
  if (tiles < 512 && K >= 4096) splits = std::min<int64_t>({(1024 + tiles - 1) / tiles, K / 1024, 256});
  if (splits <= 1) {
    void* args[] = {&g};
    HIP_TRY(hipLaunchKernel(gemm_fn(ta, tb), dim3((unsigned)tiles, 1), dim3(256), args, 0, st));
    return QTT_OK;
  }
  DBuf P;
  QTT_CHECK(dalloc(P, splits * M * N));
  g.C = P.p;
  g.ldc = N;
  g.sC = M * N;
  g.beta = 0.0;
  g.ksplit = ((K + splits - 1) / splits + kGemmK - 1) / kGemmK * kGemmK;
  splits = (K + g.ksplit - 1) / g.ksplit;
  void* args[] = {&g};
  HIP_TRY(hipLaunchKernel(gemm_fn(ta, tb), dim3((unsigned)tiles, (unsigned)splits), dim3(256), args, 0, st));
  SplitSumArgs ss{P.p, C, M, N, ldc, splits, beta};
  void* args2[] = {&ss};
  HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&split_sum_kernel), dim3(grid_for(M * N)), dim3(256), args2,
                          0, st));
  HIP_TRY(hipStreamSynchronize(st));       // P is freed on return
  return QTT_OK;
}

qtt_status_t gaussian(double* out, int64_t count, uint64_t seed, uint32_t stream_id, hipStream_t st) {
  PhiloxArgs a;
  a.out = out;
  a.count = count;
  a.seed = seed;
  a.stream = stream_id;
  void* args[] = {&a};
  HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&philox_normal_kernel), dim3(grid_for((count + 1) / 2)),
                          dim3(256), args, 0, st));
  return QTT_OK;
}

template <class Args>
qtt_status_t launch1d(const void* fn, Args a, int64_t work, hipStream_t st) {
  void* args[] = {&a};
  HIP_TRY(hipLaunchKernel(fn, dim3(grid_for(work)), dim3(256), args, 0, st));
  return QTT_OK;
}

// Thin QR of the m x n matrix Z (overwritten, row-major), m >= n: Q (m x n)
// and, when R is not null, R (n x n).  Tall-skinny Householder QR when the
// blocks fit in LDS (n <= 64, m a multiple of 64): row blocks of B rows
// (a multiple of 64, so every block has at least n rows) are factored one
// per workgroup, their stacked R_b factored by one more workgroup, and
// Q = blockdiag(Q_b) Q2, R = R2.  Otherwise one workgroup factors Z through
// global memory (qr_thin_kernel).
static const size_t kQrLdsBytes = 150 * 1024;
static int64_t qr_block_rows(int64_t n) { return (int64_t)(kQrLdsBytes / (8 * (size_t)(n + 1))) / 64 * 64; }

static qtt_status_t qr_tall(double* Z, int64_t m, int64_t n, double* Q, double* R, hipStream_t st) {
  if (m < n || n > 256 || n < 1) return fail(QTT_ERR_SHAPE, "QR of %lld x %lld", (long long)m, (long long)n);
  const int64_t B = qr_block_rows(n);
  const int64_t nb = (m + B - 1) / B;
  const bool lds = n <= 64 && m % 64 == 0 && B >= 64 && B >= n &&
                   (nb == 1 || (size_t)(nb * n) * (n + 1) * 8 <= kQrLdsBytes);
  if (!lds) {
    QrArgs a;
    memset(&a, 0, sizeof(a));
    a.A = Z;
    a.Q = Q;
    a.R = R;
    a.m = m;
    a.n = n;
    a.lda = n;
    a.ldq = n;
    void* args[] = {&a};
    HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&qr_thin_kernel), dim3(1), dim3(256), args, 0, st));
    return QTT_OK;
  }
  static bool attr = false;
  if (!attr) {
    HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&qr_block_lds_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kQrLdsBytes));
    attr = true;
  }
  const void* fn = reinterpret_cast<const void*>(&qr_block_lds_kernel);
  if (nb == 1) {
    QrBlkArgs a{Z, Q, R, m, (int32_t)n, (int32_t)m};
    void* args[] = {&a};
    HIP_TRY(hipLaunchKernel(fn, dim3(1), dim3(256), args, (size_t)m * (n + 1) * 8, st));
    return QTT_OK;
  }
  DBuf Q1, Rs, Q2;
  QTT_CHECK(dalloc(Q1, m * n));
  QTT_CHECK(dalloc(Rs, nb * n * n));
  QTT_CHECK(dalloc(Q2, nb * n * n));
  QrBlkArgs a1{Z, Q1.p, Rs.p, m, (int32_t)n, (int32_t)B};
  void* args1[] = {&a1};
  HIP_TRY(hipLaunchKernel(fn, dim3((unsigned)nb), dim3(256), args1, (size_t)B * (n + 1) * 8, st));
  QrBlkArgs a2{Rs.p, Q2.p, R, nb * n, (int32_t)n, (int32_t)(nb * n)};
  void* args2[] = {&a2};
  HIP_TRY(hipLaunchKernel(fn, dim3(1), dim3(256), args2, (size_t)(nb * n) * (n + 1) * 8, st));
  QrCombineArgs c{Q1.p, Q2.p, Q, m, (int32_t)n, (int32_t)B};
  QTT_CHECK(launch1d(reinterpret_cast<const void*>(&qr_combine_kernel), c, m * n, st));
  HIP_TRY(hipStreamSynchronize(st));       // the temporaries are freed on return
  return QTT_OK;
}

// Thin Q of the m x n matrix Z (overwritten), m >= n.
qtt_status_t qr_thin(double* Z, int64_t m, int64_t n, double* Q, hipStream_t st) {
  return qr_tall(Z, m, n, Q, nullptr, st);
}



// Smallest r >= 1 whose discarded singular values s_r, s_{r+1}, ... (sorted
// descending) have Euclidean norm <= delta (Algorithm 1's rank rule).
int keep_rank(const std::vector<double>& s, double delta) {
  const int n = (int)s.size();
  std::vector<double> tail(n + 1, 0.0);
  for (int i = n - 1; i >= 0; --i) tail[i] = tail[i + 1] + s[i] * s[i];
  int r = 1;
  while (r < n && std::sqrt(tail[r]) > delta) ++r;
  return r;
}

// Left singular vectors U (lr x c) and singular values s (c) of the
// lr x cols matrix B (row-major): for cols >= lr through the QR of B^T
// (B = R^T Q^T, so B and R^T share U and s), else of B itself; one-sided
// Jacobi on the small matrix.
qtt_status_t left_svd(const double* B, int64_t lr, int64_t cols, DBuf& U, DBuf& sv, int64_t* c_out, hipStream_t st) {
  DBuf Mb;
  const double* M = B;
  int64_t c = cols;
  if (cols >= lr) {
    DBuf Bt, Qb, R;
    QTT_CHECK(dalloc(Bt, cols * lr));
    TransposeArgs ta{B, Bt.p, 1, lr, cols};         // Bt[j][i] = B[i][j]
    QTT_CHECK(launch1d(reinterpret_cast<const void*>(&transpose_kernel), ta, cols * lr, st));
    QTT_CHECK(dalloc(Qb, cols * lr));
    QTT_CHECK(dalloc(R, lr * lr));
    QTT_CHECK(qr_tall(Bt.p, cols, lr, Qb.p, R.p, st));
    QTT_CHECK(dalloc(Mb, lr * lr));
    TransposeArgs tr{R.p, Mb.p, 1, lr, lr};          // M = R^T
    QTT_CHECK(launch1d(reinterpret_cast<const void*>(&transpose_kernel), tr, lr * lr, st));
    HIP_TRY(hipStreamSynchronize(st));
    M = Mb.p;
    c = lr;
  }
  QTT_CHECK(dalloc(U, lr * c));
  QTT_CHECK(dalloc(sv, c));
  SvdArgs sa{M, U.p, sv.p, (int32_t)lr, (int32_t)c};
  static bool attr = false;
  if (!attr) {
    HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_svd_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kEigMax * (kEigMax + 1) * 8));
    attr = true;
  }
  void* args[] = {&sa};
  HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&jacobi_svd_kernel), dim3(1), dim3(256), args,
                          (size_t)lr * (c + 1) * 8, st));
  HIP_TRY(hipStreamSynchronize(st));
  *c_out = c;
  return QTT_OK;
}

// Stage 2: t's cores 0..d-2 are left-orthonormal; truncate right to left:
// core k (as the r_{k-1} x n_k r_k matrix B) = U diag(s) W^T, keep the rank
// of Algorithm 1's rule, core k <- diag(1/s) U_r^T B, core k-1 <- core k-1
// U_r diag(s).
qtt_status_t truncate_sweep(DevTT& t, double eps, hipStream_t st, double floor = 0.0) {
  const int d = t.d;
  if (d == 1) return QTT_OK;
  // ||c|| = ||core d-1|| (everything to its left is orthonormal)
  std::vector<double> h(t.len(d - 1));
  HIP_TRY(hipMemcpyAsync(h.data(), t.core[d - 1].p, h.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double nrm = 0.0;
  for (double v : h) nrm += v * v;
  nrm = std::sqrt(nrm);
  const double delta = std::max(eps * nrm, floor) / std::sqrt((double)(d - 1));
  for (int k = d - 1; k >= 1; --k) {
    const int64_t lr = t.r[k], cols = t.n[k] * t.r[k + 1];
    if (lr > kEigMax) return fail(QTT_ERR_SHAPE, "rank %lld above %d in the truncation", (long long)lr, kEigMax);
    DBuf V, sv, U, US, sel;
    int64_t c = 0;
    QTT_CHECK(left_svd(t.core[k].p, lr, cols, V, sv, &c, st));
    std::vector<double> hs(c);
    HIP_TRY(hipMemcpy(hs.data(), sv.p, c * 8, hipMemcpyDeviceToHost));
    std::vector<int> idx(c);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return hs[x] > hs[y]; });
    std::vector<double> s(c);
    for (int i = 0; i < c; ++i) s[i] = hs[idx[i]];
    const int r = keep_rank(s, delta);
    // upload [s | 1/s | ones] and the indices
    std::vector<double> up(3 * r);
    for (int i = 0; i < r; ++i) {
      up[i] = s[i];
      up[r + i] = s[i] > 0.0 ? 1.0 / s[i] : 0.0;
      up[2 * r + i] = 1.0;
    }
    std::vector<int32_t> ix(idx.begin(), idx.begin() + r);
    QTT_CHECK(dalloc(sel, 3 * r + (r + 1) / 2 + 1));
    HIP_TRY(hipMemcpyAsync(sel.p, up.data(), up.size() * 8, hipMemcpyHostToDevice, st));
    int32_t* dix = reinterpret_cast<int32_t*>(sel.p + 3 * r);
    HIP_TRY(hipMemcpyAsync(dix, ix.data(), ix.size() * 4, hipMemcpyHostToDevice, st));
    QTT_CHECK(dalloc(U, lr * r));
    QTT_CHECK(dalloc(US, lr * r));
    // V is lr x c: select its columns (SelectArgs reads V[i * n + idx], n = c here)
    SelectArgs sa{V.p, dix, sel.p + 2 * r, U.p, (int32_t)lr, (int32_t)r};
    sa.ldv = (int32_t)c;
    QTT_CHECK(launch1d(reinterpret_cast<const void*>(&select_columns_kernel), sa, lr * r, st));
    sa.scale = sel.p;
    sa.out = US.p;
    QTT_CHECK(launch1d(reinterpret_cast<const void*>(&select_columns_kernel), sa, lr * r, st));
    // core k <- diag(1/s) U_r^T B  (r x cols)
    DBuf nk;
    QTT_CHECK(dalloc(nk, r * cols));
    QTT_CHECK(gemm(true, false, r, cols, lr, 1.0, U.p, r, t.core[k].p, cols, 0.0, nk.p, cols, st));
    ScaleRowsArgs sr{nk.p, sel.p + r, r, cols};
    QTT_CHECK(launch1d(reinterpret_cast<const void*>(&scale_rows_kernel), sr, r * cols, st));
    // core k-1 <- core k-1 U_r diag(s)
    const int64_t rows = t.r[k - 1] * t.n[k - 1];
    DBuf pk;
    QTT_CHECK(dalloc(pk, rows * r));
    QTT_CHECK(gemm(false, false, rows, r, lr, 1.0, t.core[k - 1].p, lr, US.p, r, 0.0, pk.p, r, st));
    HIP_TRY(hipStreamSynchronize(st));
    t.core[k] = std::move(nk);
    t.core[k - 1] = std::move(pk);
    t.r[k] = r;
  }
  return QTT_OK;
}

// Sketch ranks: l_k <= ell, R_k, l_{k-1} n_k, and n_{k+1} l_{k+1} (the ranks a
// TT with these modes can have at all).
std::vector<int64_t> sketch_ranks(const TTView& in, int64_t ell) {
  const int d = in.d;
  std::vector<int64_t> l(d + 1, 1);
  for (int k = 1; k < d; ++k) l[k] = std::min<int64_t>({ell, in.r[k], l[k - 1] * in.n[k - 1]});
  for (int k = d - 1; k >= 1; --k) l[k] = std::min<int64_t>(l[k], in.n[k] * l[k + 1]);
  return l;
}

// Stage 1 for a TT input with sketch ranks l; out receives left-orthonormal
// cores 0..d-2 and the last core.
qtt_status_t randomized_orthogonalize(const TTView& in, const std::vector<int64_t>& l, uint64_t seed, DevTT& out,
                                      hipStream_t st) {
  const int d = in.d;
  out.d = d;
  out.n = in.n;
  out.r = l;
  out.core.clear();
  out.core.resize(d);
  // right to left: W[k] is R_k x l_k (W[d] = 1)
  std::vector<DBuf> W(d + 1);
  QTT_CHECK(dalloc(W[d], 1));
  const double one = 1.0;
  HIP_TRY(hipMemcpyAsync(W[d].p, &one, 8, hipMemcpyHostToDevice, st));
  for (int k = d - 1; k >= 1; --k) {
    const int64_t R0 = in.r[k], n = in.n[k], R1 = in.r[k + 1];
    DBuf T, Om;
    QTT_CHECK(dalloc(T, R0 * n * l[k + 1]));
    QTT_CHECK(gemm(false, false, R0 * n, l[k + 1], R1, 1.0, in.core[k], R1, W[k + 1].p, l[k + 1], 0.0, T.p,
                   l[k + 1], st));
    QTT_CHECK(dalloc(Om, l[k] * n * l[k + 1]));
    QTT_CHECK(gaussian(Om.p, l[k] * n * l[k + 1], seed, (uint32_t)k, st));
    QTT_CHECK(dalloc(W[k], R0 * l[k]));
    QTT_CHECK(gemm(false, true, R0, l[k], n * l[k + 1], 1.0, T.p, n * l[k + 1], Om.p, n * l[k + 1], 0.0, W[k].p,
                   l[k], st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  // left to right: Y is (l_{k-1} n_k) x R_k
  DBuf Y;
  const double* Yp = in.core[0];
  for (int k = 0; k < d - 1; ++k) {
    const int64_t rows = l[k] * in.n[k], R1 = in.r[k + 1];
    DBuf Z;
    QTT_CHECK(dalloc(Z, rows * l[k + 1]));
    QTT_CHECK(gemm(false, false, rows, l[k + 1], R1, 1.0, Yp, R1, W[k + 1].p, l[k + 1], 0.0, Z.p, l[k + 1], st));
    QTT_CHECK(dalloc(out.core[k], rows * l[k + 1]));
    QTT_CHECK(qr_thin(Z.p, rows, l[k + 1], out.core[k].p, st));
    DBuf M;
    QTT_CHECK(dalloc(M, l[k + 1] * R1));
    QTT_CHECK(gemm(true, false, l[k + 1], R1, rows, 1.0, out.core[k].p, l[k + 1], Yp, R1, 0.0, M.p, R1, st));
    const int64_t n1 = in.n[k + 1], R2 = in.r[k + 2];
    DBuf Yn;
    QTT_CHECK(dalloc(Yn, l[k + 1] * n1 * R2));
    QTT_CHECK(gemm(false, false, l[k + 1], n1 * R2, R1, 1.0, M.p, R1, in.core[k + 1], n1 * R2, 0.0, Yn.p, n1 * R2,
                   st));
    HIP_TRY(hipStreamSynchronize(st));
    Y = std::move(Yn);
    Yp = Y.p;
    W[k + 1].reset();
  }
  const int64_t last = l[d - 1] * in.n[d - 1];
  QTT_CHECK(dalloc(out.core[d - 1], last));
  HIP_TRY(hipMemcpyAsync(out.core[d - 1].p, Yp, last * 8, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return QTT_OK;
}

// Whether the kept ranks leave room below the sketch ranks wherever the
// sketch rank was below what the input could hold.
bool sketch_enough(const TTView& in, const std::vector<int64_t>& l, const std::vector<int64_t>& kept,
                   int64_t ell) {
  const std::vector<int64_t> full = sketch_ranks(in, INT64_MAX / 4);
  for (int k = 1; k < in.d; ++k) {
    if (l[k] >= full[k]) continue;              // the sketch holds the whole range there
    const int64_t margin = std::max<int64_t>(4, l[k] / 8);
    if (kept[k] > l[k] - margin && l[k] >= ell) return false;
  }
  return true;
}

// Rounding with the sketch rank grown until it leaves room (or reaches
// max_rank: *capped is then set).  floor > 0: accuracy max(eps ||c||, floor).
qtt_status_t round_tt(const TTView& in, double eps, int64_t max_rank, uint64_t seed, DevTT& out, hipStream_t st,
                      bool* capped, double floor = 0.0) {
  *capped = false;
  const int d = in.d;
  if (d == 1) {
    out.d = 1;
    out.n = in.n;
    out.r = in.r;
    out.core.clear();
    out.core.resize(1);
    QTT_CHECK(dalloc(out.core[0], in.n[0]));
    HIP_TRY(hipMemcpyAsync(out.core[0].p, in.core[0], in.n[0] * 8, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return QTT_OK;
  }
  int64_t ell = std::min<int64_t>(max_rank, 32);
  for (;;) {
    const std::vector<int64_t> l = sketch_ranks(in, ell);
    QTT_CHECK(randomized_orthogonalize(in, l, seed, out, st));
    QTT_CHECK(truncate_sweep(out, eps, st, floor));
    if (sketch_enough(in, l, out.r, ell)) return QTT_OK;
    if (ell >= max_rank) {
      *capped = true;
      return QTT_OK;
    }
    ell = std::min<int64_t>(2 * ell, max_rank);
  }
}

// Stage 1 for a full vector x (length prod n): randomized TT-SVD, the
// remainder M (l_{k-1} x C_{k-1}, columns (i_k, i_{k+1}, ...) first digit
// fastest) sketched by a Gaussian C_k x l_k matrix.
qtt_status_t randomized_compress(const double* x, const std::vector<int64_t>& n, int64_t ell, uint64_t seed,
                                 DevTT& out, std::vector<int64_t>& l, hipStream_t st) {
  const int d = (int)n.size();
  out.d = d;
  out.n = n;
  out.core.clear();
  out.core.resize(d);
  l.assign(d + 1, 1);
  int64_t C = 1;
  for (auto v : n) C *= v;
  DBuf Mb;
  const double* M = x;
  for (int k = 0; k < d - 1; ++k) {
    const int64_t nk = n[k];
    C /= nk;                                           // columns after this mode
    l[k + 1] = std::min<int64_t>({ell, l[k] * nk, C});
    const int64_t rows = l[k] * nk;
    // Yt[(a, i_k)][q] = M[a][q][i_k]
    DBuf Yt;
    QTT_CHECK(dalloc(Yt, rows * C));
    TransposeArgs ta{M, Yt.p, l[k], C, nk};
    QTT_CHECK(launch1d(reinterpret_cast<const void*>(&transpose_kernel), ta, rows * C, st));
    DBuf Om, Z;
    QTT_CHECK(dalloc(Om, C * l[k + 1]));
    QTT_CHECK(gaussian(Om.p, C * l[k + 1], seed, (uint32_t)(1000 + k), st));
    QTT_CHECK(dalloc(Z, rows * l[k + 1]));
    QTT_CHECK(gemm(false, false, rows, l[k + 1], C, 1.0, Yt.p, C, Om.p, l[k + 1], 0.0, Z.p, l[k + 1], st));
    QTT_CHECK(dalloc(out.core[k], rows * l[k + 1]));
    QTT_CHECK(qr_thin(Z.p, rows, l[k + 1], out.core[k].p, st));
    DBuf Mn;
    QTT_CHECK(dalloc(Mn, l[k + 1] * C));
    QTT_CHECK(gemm(true, false, l[k + 1], C, rows, 1.0, out.core[k].p, l[k + 1], Yt.p, C, 0.0, Mn.p, C, st));
    HIP_TRY(hipStreamSynchronize(st));
    Mb = std::move(Mn);
    M = Mb.p;
  }
  const int64_t last = l[d - 1] * n[d - 1];
  QTT_CHECK(dalloc(out.core[d - 1], last));
  HIP_TRY(hipMemcpyAsync(out.core[d - 1].p, M, last * 8, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  out.r = l;
  return QTT_OK;
}

qtt_status_t check_tt_args(int32_t d, const int64_t* n, const int64_t* ranks, int32_t max_rank, double eps) {
  if (d < 1 || d > 64 || !n) return fail(QTT_ERR_INVALID_ARG, "d = %d outside [1, 64] or null modes", d);
  for (int k = 0; k < d; ++k)
    if (n[k] < 1) return fail(QTT_ERR_SHAPE, "mode %d < 1", k);
  if (ranks) {
    if (ranks[0] != 1 || ranks[d] != 1) return fail(QTT_ERR_SHAPE, "boundary ranks must be 1");
    for (int k = 1; k < d; ++k)
      if (ranks[k] < 1) return fail(QTT_ERR_SHAPE, "rank %d < 1", k);
  }
  if (max_rank < 1 || max_rank > kEigMax) return fail(QTT_ERR_INVALID_ARG, "max_rank outside [1, %d]", kEigMax);
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(QTT_ERR_INVALID_ARG, "eps must be finite and >= 0");
  return QTT_OK;
}

// Copy a rounded TT into caller buffers and report its ranks.
qtt_status_t export_tt(const DevTT& t, double* const* out, int64_t* out_ranks, hipStream_t st) {
  for (int k = 0; k < t.d; ++k) {
    if (!out[k]) return fail(QTT_ERR_INVALID_ARG, "output core %d is null", k);
    HIP_TRY(hipMemcpyAsync(out[k], t.core[k].p, t.len(k) * 8, hipMemcpyDeviceToDevice, st));
  }
  for (int k = 0; k <= t.d; ++k) out_ranks[k] = t.r[k];
  HIP_TRY(hipStreamSynchronize(st));
  return QTT_OK;
}

// Cores of the QTT matrix product A B (A's rank fastest in each merged index),
// as TT cores with mode m_k n_k.
qtt_status_t matmul_tt(const TTView& A, const std::vector<int64_t>& m, const std::vector<int64_t>& l,
                       const TTView& B, const std::vector<int64_t>& n, DevTT& C, hipStream_t st) {
  const int d = A.d;
  C.d = d;
  C.n.resize(d);
  C.r.resize(d + 1);
  C.core.clear();
  C.core.resize(d);
  for (int k = 0; k <= d; ++k) C.r[k] = A.r[k] * B.r[k];
  for (int k = 0; k < d; ++k) {
    C.n[k] = m[k] * n[k];
    MatmulCoresArgs a;
    a.A = A.core[k];
    a.B = B.core[k];
    a.ra0 = A.r[k];
    a.ra1 = A.r[k + 1];
    a.rb0 = B.r[k];
    a.rb1 = B.r[k + 1];
    a.m = m[k];
    a.l = l[k];
    a.n = n[k];
    a.total = C.len(k);
    QTT_CHECK(dalloc(C.core[k], a.total));
    a.C = C.core[k].p;
    QTT_CHECK(launch1d(reinterpret_cast<const void*>(&matmul_cores_kernel), a, a.total, st));
  }
  return QTT_OK;
}

// Cores of sum_t c_t X_t (TT sum: ranks add; c_t scales the first core).
qtt_status_t lincomb_tt(const std::vector<std::pair<double, TTView>>& terms, DevTT& out, hipStream_t st) {
  const TTView& f = terms[0].second;
  const int d = f.d;
  out.d = d;
  out.n = f.n;
  out.r.assign(d + 1, 0);
  out.r[0] = out.r[d] = 1;
  for (int k = 1; k < d; ++k)
    for (auto& t : terms) out.r[k] += t.second.r[k];
  out.core.clear();
  out.core.resize(d);
  for (int k = 0; k < d; ++k) {
    QTT_CHECK(dalloc(out.core[k], out.len(k)));
    HIP_TRY(hipMemsetAsync(out.core[k].p, 0, out.len(k) * 8, st));
    int64_t o0 = 0, o1 = 0;
    for (auto& t : terms) {
      const TTView& v = t.second;
      BlockCopyArgs b;
      b.src = v.core[k];
      b.dst = out.core[k].p;
      b.r0 = v.r[k];
      b.n = v.n[k];
      b.r1 = v.r[k + 1];
      b.R1 = out.r[k + 1];
      b.off0 = (k == 0) ? 0 : o0;
      b.off1 = (k == d - 1) ? 0 : o1;
      b.scale = (k == 0) ? t.first : 1.0;
      QTT_CHECK(launch1d(reinterpret_cast<const void*>(&block_copy_kernel), b, b.r0 * b.n * b.r1, st));
      o0 += v.r[k];
      o1 += v.r[k + 1];
    }
  }
  return QTT_OK;
}

double tt_norm_first_core(const DevTT& t, hipStream_t st) {
  // after truncate_sweep the cores right of the first are right-orthonormal
  std::vector<double> h(t.len(0));
  if (hipMemcpyAsync(h.data(), t.core[0].p, h.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess) return NAN;
  if (hipStreamSynchronize(st) != hipSuccess) return NAN;
  double s = 0.0;
  for (double v : h) s += v * v;
  return std::sqrt(s);
}

}  // namespace

extern "C" {

qtt_status_t qtt_tt_round(int32_t d, const int64_t* n, const int64_t* ranks, const double* const* cores,
                          double eps, int32_t max_rank, uint64_t seed, double* const* out, int64_t* out_ranks,
                          void* stream) {
  QTT_CHECK(check_tt_args(d, n, ranks, max_rank, eps));
  if (!ranks || !cores || !out || !out_ranks) return fail(QTT_ERR_INVALID_ARG, "null argument");
  TTView in;
  in.d = d;
  in.n.assign(n, n + d);
  in.r.assign(ranks, ranks + d + 1);
  for (int k = 0; k < d; ++k) {
    if (!cores[k]) return fail(QTT_ERR_INVALID_ARG, "core %d is null", k);
    in.core.push_back(cores[k]);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  DevTT t;
  bool capped = false;
  QTT_CHECK(round_tt(in, eps, max_rank, seed, t, st, &capped));
  QTT_CHECK(export_tt(t, out, out_ranks, st));
  if (capped) return fail(QTT_ERR_RANK, "the tolerance needs ranks above max_rank = %d", max_rank);
  return QTT_OK;
}

qtt_status_t qtt_tt_compress(int32_t d, const int64_t* n, const double* x, double eps, int32_t max_rank,
                             uint64_t seed, double* const* out, int64_t* out_ranks, void* stream) {
  QTT_CHECK(check_tt_args(d, n, nullptr, max_rank, eps));
  if (!x || !out || !out_ranks) return fail(QTT_ERR_INVALID_ARG, "null argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int64_t> nv(n, n + d);
  DevTT t;
  int64_t ell = std::min<int64_t>(max_rank, 32);
  bool capped = false;
  for (;;) {
    std::vector<int64_t> l;
    QTT_CHECK(randomized_compress(x, nv, ell, seed, t, l, st));
    QTT_CHECK(truncate_sweep(t, eps, st));
    // room check against the ranks a vector of these modes can have
    TTView full;
    full.d = d;
    full.n = nv;
    full.r.assign(d + 1, INT64_MAX / 4);
    full.r[0] = full.r[d] = 1;
    if (d == 1 || sketch_enough(full, l, t.r, ell)) break;
    if (ell >= max_rank) {
      capped = true;
      break;
    }
    ell = std::min<int64_t>(2 * ell, max_rank);
  }
  QTT_CHECK(export_tt(t, out, out_ranks, st));
  if (capped) return fail(QTT_ERR_RANK, "the tolerance needs ranks above max_rank = %d", max_rank);
  return QTT_OK;
}

qtt_status_t qtt_matrix_cores(qtt_matrix_t A, double* const* host_cores) {
  if (!A || A->d < 1 || !host_cores) return fail(QTT_ERR_INVALID_ARG, "null handle or output");
  if (!(A->dtypes & QTT_FP64)) return fail(QTT_ERR_DTYPE, "the handle holds no FP64 copy");
  for (int k = 0; k < A->d; ++k) {
    const CoreDev& c = A->core[k];
    if (!host_cores[k]) return fail(QTT_ERR_INVALID_ARG, "output core %d is null", k);
    HIP_TRY(hipMemcpy(host_cores[k], c.g64, (size_t)c.r_in * c.m * c.n * c.r_out * 8, hipMemcpyDeviceToHost));
  }
  return QTT_OK;
}

qtt_status_t qtt_invert_newton_schulz(qtt_matrix_t A, qtt_matrix_t X0, double eps, int32_t max_rank,
                                      int32_t max_iter, double tol, double theta, uint64_t seed, uint32_t dtypes,
                                      qtt_matrix_t* Xinv, double* history, int32_t* steps, void* stream) {
  if (!A || !X0 || !Xinv || A->d < 1) return fail(QTT_ERR_INVALID_ARG, "null handle or output");
  *Xinv = nullptr;
  if (!(A->dtypes & QTT_FP64) || !(X0->dtypes & QTT_FP64))
    return fail(QTT_ERR_DTYPE, "A and X0 need their FP64 copies");
  if (A->d != X0->d) return fail(QTT_ERR_SHAPE, "A and X0 have different core counts");
  for (int k = 0; k < A->d; ++k)
    if (A->m[k] != A->n[k] || X0->m[k] != A->m[k] || X0->n[k] != A->n[k])
      return fail(QTT_ERR_SHAPE, "inversion needs square, identical modes (core %d)", k);
  if (max_iter < 0 || !(tol >= 0.0) || !(theta >= 0.0) || !std::isfinite(theta))
    return fail(QTT_ERR_INVALID_ARG, "bad max_iter, tol or theta");
  QTT_CHECK(check_tt_args(A->d, A->m.data(), nullptr, max_rank, eps));
  if (dtypes == 0 || (dtypes & ~7u)) return fail(QTT_ERR_INVALID_ARG, "dtypes must be an OR of QTT_FP64/FP32/BF16");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int d = A->d;
  std::vector<int64_t> m = A->m, mm(d);
  for (int k = 0; k < d; ++k) mm[k] = m[k] * m[k];
  auto handle_view = [&](const qtt_matrix_s* H) {
    TTView v;
    v.d = d;
    v.n = mm;
    v.r = H->ranks;
    for (auto& c : H->core) v.core.push_back(c.g64);
    return v;
  };
  const TTView Av = handle_view(A);
  // identity cores delta(i, j), rank 1
  DevTT Id;
  Id.d = d;
  Id.n = mm;
  Id.r.assign(d + 1, 1);
  Id.core.resize(d);
  for (int k = 0; k < d; ++k) {
    std::vector<double> h(mm[k], 0.0);
    for (int64_t i = 0; i < m[k]; ++i) h[i * m[k] + i] = 1.0;
    QTT_CHECK(dalloc(Id.core[k], mm[k]));
    HIP_TRY(hipMemcpyAsync(Id.core[k].p, h.data(), mm[k] * 8, hipMemcpyHostToDevice, st));
  }
  // X <- X0
  DevTT X;
  X.d = d;
  X.n = mm;
  X.r = X0->ranks;
  X.core.resize(d);
  for (int k = 0; k < d; ++k) {
    QTT_CHECK(dalloc(X.core[k], X.len(k)));
    HIP_TRY(hipMemcpyAsync(X.core[k].p, X0->core[k].g64, X.len(k) * 8, hipMemcpyDeviceToDevice, st));
  }
  double ident = 1.0;
  for (int k = 0; k < d; ++k) ident *= (double)m[k];
  ident = std::sqrt(ident);
  bool capped_any = false;
  int t = 0;
  for (;; ++t) {
    DevTT AX, AXr, R, Rr;
    bool cap = false;
    QTT_CHECK(matmul_tt(Av, m, m, view(X), m, AX, st));
    QTT_CHECK(round_tt(view(AX), eps, max_rank, seed + 4 * t, AXr, st, &cap));
    capped_any |= cap;
    AX = DevTT();
    QTT_CHECK(lincomb_tt({{1.0, view(Id)}, {-1.0, view(AXr)}}, R, st));
    // R is rounded against the scale of I (X's accuracy), not its own norm
    QTT_CHECK(round_tt(view(R), eps, max_rank, seed + 4 * t + 1, Rr, st, &cap, eps * ident));
    capped_any |= cap;
    const double h = tt_norm_first_core(Rr, st) / ident;
    if (history) history[t] = h;
    if (!std::isfinite(h)) return fail(QTT_ERR_NONFINITE, "residual of step %d is not finite", t);
    if (h <= tol || t >= max_iter) break;
    // the next iterate is within about h^2 of the inverse: theta > 0 rounds
    // it (and 2 I - A X) no finer than that
    const double tau = std::max(eps, theta * h * h);
    DevTT Z, Zr, XZ, Xn;
    QTT_CHECK(lincomb_tt({{1.0, view(Id)}, {1.0, view(Rr)}}, Z, st));      // 2 I - A X = I + R
    QTT_CHECK(round_tt(view(Z), tau, max_rank, seed + 4 * t + 2, Zr, st, &cap));
    capped_any |= cap;
    QTT_CHECK(matmul_tt(view(X), m, m, view(Zr), m, XZ, st));
    QTT_CHECK(round_tt(view(XZ), tau, max_rank, seed + 4 * t + 3, Xn, st, &cap));
    capped_any |= cap;
    X = std::move(Xn);
  }
  if (steps) *steps = t;
  // the inverse as a handle: cores back to the host, loaded like any matrix
  std::vector<std::vector<double>> hc(d);
  std::vector<const double*> ptrs(d);
  for (int k = 0; k < d; ++k) {
    hc[k].resize(X.len(k));
    HIP_TRY(hipMemcpyAsync(hc[k].data(), X.core[k].p, X.len(k) * 8, hipMemcpyDeviceToHost, st));
    ptrs[k] = hc[k].data();
  }
  HIP_TRY(hipStreamSynchronize(st));
  QTT_CHECK(qtt_matrix_load(d, X.r.data(), m.data(), m.data(), ptrs.data(), dtypes, Xinv));
  if (capped_any) return fail(QTT_ERR_RANK, "a rounding needed ranks above max_rank = %d", max_rank);
  return QTT_OK;
}

}  // extern "C"
