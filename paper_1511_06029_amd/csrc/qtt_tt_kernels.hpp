// Device kernels of the TT-format operations of libqtt: rounding of a tensor
// given in TT form (the decomposition Algorithm 1, section 2.3, gives for the
// tensor the cores represent), compression of a full vector, and the QTT
// matrix product used by the Newton-Hotelling-Schulz inversion.
//
// All of it is FP64 dense linear algebra on small or skinny matrices:
//   * gemm_kernel        C = alpha op(A) op(B) + beta C, row-major, batched;
//   * philox_normal_kernel  N(0,1) sketch entries from a counter-based
//                        generator (Philox4x32-10, Salmon, Moraes, Dror and
//                        Shaw, SC'11) with the Box-Muller transform;
//   * qr_thin_kernel     Householder QR of one m x n matrix (m >= n) per
//                        workgroup, giving the thin Q;
//   * qr_block_lds_kernel, qr_combine_kernel  the same QR as a tall-skinny
//                        QR: row blocks factored in LDS, one per workgroup,
//                        then their stacked R factors, Q recombined;
//   * jacobi_svd_kernel  singular values and left singular vectors of one
//                        m x c matrix (c <= m <= 128) per workgroup,
//                        one-sided Jacobi in round-robin order, in LDS;
//   * matmul_cores_kernel  the cores of a QTT matrix product (ranks multiply);
//   * block_copy_kernel  places a scaled core into a block of a larger core
//                        (the cores of a TT sum).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtt {

// ---------------------------------------------------------------------------
// GEMM.  op(A) is M x K: A[i * lda + k], or A[k * lda + i] when TA.  op(B) is
// K x N: B[k * ldb + j], or B[j * ldb + k] when TB.  C[i * ldc + j].  Batch b
// (blockIdx.y) offsets the three pointers by sA, sB, sC.  Tiles of 64 x 64
// outputs, 256 threads each owning a 4 x 4 block, contraction in chunks of 16
// staged in LDS (k-major, so every thread reads its four rows and four
// columns as contiguous runs).
// ---------------------------------------------------------------------------
struct GemmArgs {
  const double* A;
  const double* B;
  double* C;
  int64_t M, N, K;
  int64_t lda, ldb, ldc;
  int64_t sA, sB, sC;
  int64_t tiles_n;      // column tiles (N / 64 rounded up)
  int64_t ksplit;       // > 0: split of the contraction blockIdx.y works on
                        // (indices [y ksplit, min(K, (y + 1) ksplit)), C + y sC)
  double alpha, beta;
};

constexpr int kGemmT = 64, kGemmK = 16;

template <bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_kernel(const GemmArgs a) {
  __shared__ double As[kGemmK][kGemmT + 2];
  __shared__ double Bs[kGemmK][kGemmT + 2];
  const int tid = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t m0 = (tile / a.tiles_n) * kGemmT, n0 = (tile % a.tiles_n) * kGemmT;
  const double* A = a.A + (int64_t)blockIdx.y * a.sA;
  const double* B = a.B + (int64_t)blockIdx.y * a.sB;
  double* C = a.C + (int64_t)blockIdx.y * a.sC;
  const int64_t kbeg = a.ksplit > 0 ? (int64_t)blockIdx.y * a.ksplit : 0;
  const int64_t kend = a.ksplit > 0 ? (kbeg + a.ksplit < a.K ? kbeg + a.ksplit : a.K) : a.K;
  const int ty = tid >> 4, tx = tid & 15;   // rows 4 ty .. 4 ty + 3, columns 4 tx .. 4 tx + 3
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kGemmK) {
    // A tile: 64 rows x 16 contraction indices, 4 values per thread
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int i, kk;
      if (TA) { kk = tid >> 4; i = (tid & 15) * 4 + e; }   // consecutive i along memory
      else { i = tid >> 2; kk = (tid & 3) * 4 + e; }         // consecutive k along memory
      const int64_t gi = m0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < a.M && gk < kend) v = TA ? A[gk * a.lda + gi] : A[gi * a.lda + gk];
      As[kk][i] = v;
    }
    // B tile: 16 contraction indices x 64 columns
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int j, kk;
      if (TB) { j = tid >> 2; kk = (tid & 3) * 4 + e; }
      else { kk = tid >> 4; j = (tid & 15) * 4 + e; }
      const int64_t gj = n0 + j, gk = k0 + kk;
      double v = 0.0;
      if (gj < a.N && gk < kend) v = TB ? B[gj * a.ldb + gk] : B[gk * a.ldb + gj];
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGemmK; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = As[kk][4 * ty + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = Bs[kk][4 * tx + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t gi = m0 + 4 * ty + r;
    if (gi >= a.M) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t gj = n0 + 4 * tx + c;
      if (gj >= a.N) continue;
      double* p = C + gi * a.ldc + gj;
      *p = a.beta == 0.0 ? a.alpha * acc[r][c] : a.alpha * acc[r][c] + a.beta * *p;
    }
  }
}

// C[i ldc + j] = sum_s P[s][i N + j] + beta C[i ldc + j]: the partial products
// of a split contraction, added in split order.
struct SplitSumArgs {
  const double* P;
  double* C;
  int64_t M, N, ldc, splits;
  double beta;
};

__global__ void __launch_bounds__(256) split_sum_kernel(const SplitSumArgs a) {
  const int64_t MN = a.M * a.N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < MN; e += (int64_t)gridDim.x * 256) {
    double t = 0.0;
    for (int64_t s2 = 0; s2 < a.splits; ++s2) t += a.P[s2 * MN + e];
    double* c = a.C + (e / a.N) * a.ldc + e % a.N;
    *c = a.beta == 0.0 ? t : t + a.beta * *c;
  }
}

// ---------------------------------------------------------------------------
// Philox4x32-10 and Box-Muller: element e of the array is normal number
// (e mod 2) of the pair made from the block with counter (e / 2, stream).
// ---------------------------------------------------------------------------
struct PhiloxArgs {
  double* out;
  int64_t count;
  uint64_t seed;
  uint32_t stream;
};

__device__ inline void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint64_t p0 = (uint64_t)M0 * c[0], p1 = (uint64_t)M1 * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k0, k1);
    k0 += W0;
    k1 += W1;
  }
}

__global__ void __launch_bounds__(256) philox_normal_kernel(const PhiloxArgs a) {
  const int64_t npair = (a.count + 1) / 2;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npair; p += (int64_t)gridDim.x * 256) {
    uint32_t c[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), a.stream, 0u};
    philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    // two uniforms in (0, 1] with 64 random bits each
    const double two64 = 5.421010862427522e-20;   // 2^-64
    const double u1 = ((double)(((uint64_t)c[0] << 32) | c[1]) + 1.0) * two64;
    const double u2 = (double)(((uint64_t)c[2] << 32) | c[3]) * two64;
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586 * u2;
    a.out[2 * p] = rad * cos(ang);
    if (2 * p + 1 < a.count) a.out[2 * p + 1] = rad * sin(ang);
  }
}

// ---------------------------------------------------------------------------
// Householder QR of one m x n matrix (row-major, lda), m >= n, n <= 256, per
// workgroup; A is overwritten by the Householder vectors, Q (m x n, ldq)
// receives the thin orthonormal factor and R (n x n, row-major, if not NULL)
// the triangular one.  Column j: v = x - alpha e_1 with alpha = -sign(x_0)
// ||x||, H_j = I - beta v v^T, beta = 2 / ||v||^2 (0 for a zero v); R_jj =
// alpha, R_jc (c > j) = row j after step j.  Q = H_0 H_1 ... H_{n-1}
// [I_n; 0], formed backwards.
// ---------------------------------------------------------------------------
struct QrArgs {
  double* A;
  double* Q;
  double* R;
  int64_t m, n, lda, ldq;
  int64_t sA, sQ;     // batch strides (blockIdx.x)
};

__device__ inline double block_sum256(double v, double* red) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  const double s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// Householder QR of one row block per workgroup with the block in LDS
// (rows x (n + 1) doubles, n <= 64): the same reflectors as qr_thin_kernel
// (x0 - alpha, alpha = -sign(x0) ||x||), R_b (n x n) written out, then the
// thin Q_b formed in place by accumulating the reflectors from the last to
// the first (column j of Q is H_0 .. H_j e_j).  Block b holds rows
// [b B, min(m, (b + 1) B)); every block has at least n rows (host).  Used
// for both levels of the tall-skinny QR: the blocks of Z, then the stacked
// R_b (one block).
// ---------------------------------------------------------------------------
struct QrBlkArgs {
  const double* A;     // m x n, row-major (leading dimension n)
  double* Q;           // m x n, the same rows
  double* R;           // (blocks) x n x n, block b at b n n; may be null
  int64_t m;
  int32_t n, B;
};

__global__ void __launch_bounds__(256) qr_block_lds_kernel(const QrBlkArgs a) {
  extern __shared__ double As[];
  __shared__ double red[4];
  __shared__ double beta_s[64];
  __shared__ double alpha_s[64];
  __shared__ double part[256];
  __shared__ double w[64];
  const int tid = threadIdx.x;
  const int n = a.n, ld = n + 1;
  const int64_t r0 = (int64_t)blockIdx.x * a.B;
  const int mb = (int)((a.m - r0 < a.B) ? a.m - r0 : a.B);
  for (int e = tid; e < mb * n; e += 256) {
    const int i = e / n, c = e - (e / n) * n;
    As[i * ld + c] = a.A[(r0 + i) * n + c];
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double ss = 0.0;
    for (int i = j + tid; i < mb; i += 256) ss += As[i * ld + j] * As[i * ld + j];
    const double s = block_sum256(ss, red);
    const double x0 = As[j * ld + j];
    const double nrm = sqrt(s);
    const double alpha = (x0 >= 0.0) ? -nrm : nrm;
    const double v0 = x0 - alpha;
    const double vn2 = s - x0 * x0 + v0 * v0;
    const double beta = (vn2 > 0.0) ? 2.0 / vn2 : 0.0;
    __syncthreads();
    if (tid == 0) {
      As[j * ld + j] = v0;
      beta_s[j] = beta;
      alpha_s[j] = (vn2 > 0.0) ? alpha : x0;
    }
    __syncthreads();
    const int nc = n - 1 - j;
    if (nc > 0 && beta != 0.0) {
      // w_c = v^T A[j:, c], row groups of the 256 threads per column
      const int Gc = 256 / nc, g = tid / nc, cl = tid - (tid / nc) * nc;
      double acc = 0.0;
      if (g < Gc)
        for (int i = j + g; i < mb; i += Gc) acc += As[i * ld + j] * As[i * ld + j + 1 + cl];
      part[tid] = acc;
      __syncthreads();
      if (tid < nc) {
        double t = 0.0;
        for (int q = 0; q < Gc; ++q) t += part[q * nc + tid];
        w[tid] = t;
      }
      __syncthreads();
      for (int e = tid; e < (mb - j) * nc; e += 256) {
        const int i = j + e / nc, c2 = e - (e / nc) * nc;
        As[i * ld + j + 1 + c2] -= beta * As[i * ld + j] * w[c2];
      }
      __syncthreads();
    }
  }
  if (a.R) {
    double* R = a.R + (int64_t)blockIdx.x * n * n;
    for (int e = tid; e < n * n; e += 256) {
      const int i = e / n, c = e - (e / n) * n;
      R[e] = (c > i) ? As[i * ld + c] : (c == i ? alpha_s[i] : 0.0);
    }
  }
  __syncthreads();
  // Q in place, from the last reflector to the first: the columns c > j
  // already hold H_{j+1} .. H_{n-1} e_c (zero in rows <= j); H_j is applied
  // to them with v still in column j, which then becomes H_j e_j
  for (int j = n - 1; j >= 0; --j) {
    const double beta = beta_s[j];
    const double v0 = As[j * ld + j];
    const int nc = n - 1 - j;
    if (nc > 0 && beta != 0.0) {
      const int Gc = 256 / nc, g = tid / nc, cl = tid - (tid / nc) * nc;
      double acc = 0.0;
      if (g < Gc)
        for (int i = j + g; i < mb; i += Gc) acc += (i == j ? v0 : As[i * ld + j]) * As[i * ld + j + 1 + cl];
      part[tid] = acc;
      __syncthreads();
      if (tid < nc) {
        double t = 0.0;
        for (int q = 0; q < Gc; ++q) t += part[q * nc + tid];
        w[tid] = t;
      }
      __syncthreads();
      for (int e = tid; e < (mb - j) * nc; e += 256) {
        const int i = j + e / nc, c2 = e - (e / nc) * nc;
        As[i * ld + j + 1 + c2] -= beta * (i == j ? v0 : As[i * ld + j]) * w[c2];
      }
      __syncthreads();
    }
    for (int i = tid; i < mb; i += 256) {
      const double vi = As[i * ld + j];
      As[i * ld + j] = (i < j) ? 0.0 : (i == j ? 1.0 - beta * v0 * v0 : -beta * v0 * vi);
    }
    __syncthreads();
  }
  for (int e = tid; e < mb * n; e += 256) {
    const int i = e / n, c = e - (e / n) * n;
    a.Q[(r0 + i) * n + c] = As[i * ld + c];
  }
}

// Q = blockdiag(Q_1, .., Q_nb) Q2 for the tall-skinny QR: row i of block
// b = i div B times rows b n .. b n + n - 1 of Q2.
struct QrCombineArgs {
  const double* Q1;    // m x n
  const double* Q2;    // nb n x n
  double* Q;           // m x n
  int64_t m;
  int32_t n, B;
};

__global__ void __launch_bounds__(256) qr_combine_kernel(const QrCombineArgs a) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.m * a.n) return;
  const int n = a.n;
  const int64_t i = e / n;
  const int c = (int)(e - i * n);
  const int64_t b = i / a.B;
  const double* q1 = a.Q1 + i * n;
  const double* q2 = a.Q2 + b * n * n + c;
  double t = 0.0;
  for (int k = 0; k < n; ++k) t += q1[k] * q2[(int64_t)k * n];
  a.Q[e] = t;
}

__global__ void __launch_bounds__(256) qr_thin_kernel(const QrArgs a) {
  __shared__ double red[4];
  __shared__ double beta_s[256];
  __shared__ double alpha_s[256];
  __shared__ double part[256];
  __shared__ double w[256];
  const int tid = threadIdx.x;
  double* A = a.A + (int64_t)blockIdx.x * a.sA;
  double* Q = a.Q + (int64_t)blockIdx.x * a.sQ;
  const int64_t m = a.m, n = a.n, lda = a.lda;
  for (int64_t j = 0; j < n; ++j) {
    double ss = 0.0;
    for (int64_t i = j + tid; i < m; i += 256) ss += A[i * lda + j] * A[i * lda + j];
    const double s = block_sum256(ss, red);
    const double x0 = A[j * lda + j];
    const double nrm = sqrt(s);
    const double alpha = (x0 >= 0.0) ? -nrm : nrm;
    const double v0 = x0 - alpha;
    const double vn2 = s - x0 * x0 + v0 * v0;
    const double beta = (vn2 > 0.0) ? 2.0 / vn2 : 0.0;
    __syncthreads();
    if (tid == 0) {
      A[j * lda + j] = v0;
      beta_s[j] = beta;
      alpha_s[j] = (vn2 > 0.0) ? alpha : x0;
    }
    __syncthreads();
    const int64_t nc = n - 1 - j;
    if (nc > 0 && beta != 0.0) {
      // w_c = v^T A[j:, c], split over row groups, 256 columns at a time
      for (int64_t c0 = 0; c0 < nc; c0 += 256) {
        const int64_t cc = (nc - c0 < 256) ? nc - c0 : 256;
        const int g = (int)(tid / cc), cl = (int)(tid % cc);
        const int Gc = (int)(256 / cc);
        double acc = 0.0;
        if (g < Gc) {
          const int64_t c = j + 1 + c0 + cl;
          for (int64_t i = j + g; i < m; i += Gc) acc += A[i * lda + j] * A[i * lda + c];
        }
        part[tid] = acc;
        __syncthreads();
        if (tid < cc) {
          double t = 0.0;
          for (int q = 0; q < Gc; ++q) t += part[q * cc + tid];
          w[tid] = t;
        }
        __syncthreads();
        // A[i][c] -= beta v_i w_c for the columns of this group
        for (int64_t e = tid; e < (m - j) * cc; e += 256) {
          const int64_t i = j + e / cc, cl2 = e % cc;
          A[i * lda + j + 1 + c0 + cl2] -= beta * A[i * lda + j] * w[cl2];
        }
        __syncthreads();
      }
    }
  }
  if (a.R) {
    for (int64_t e = tid; e < n * n; e += 256) {
      const int64_t i = e / n, c = e % n;
      a.R[e] = (c > i) ? A[i * lda + c] : (c == i ? alpha_s[i] : 0.0);
    }
  }
  // Q = [I_n; 0], then the reflectors from the last to the first
  for (int64_t e = tid; e < m * n; e += 256) {
    const int64_t i = e / n, c = e % n;
    Q[i * a.ldq + c] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int64_t j = n - 1; j >= 0; --j) {
    const double beta = beta_s[j];
    if (beta == 0.0) continue;
    const int64_t nc = n - j;   // columns j .. n-1 can be touched
    for (int64_t c0 = 0; c0 < nc; c0 += 256) {
      const int64_t cc = (nc - c0 < 256) ? nc - c0 : 256;
      const int g = (int)(tid / cc), cl = (int)(tid % cc);
      const int Gc = (int)(256 / cc);
      double acc = 0.0;
      if (g < Gc) {
        const int64_t c = j + c0 + cl;
        for (int64_t i = j + g; i < m; i += Gc) acc += A[i * lda + j] * Q[i * a.ldq + c];
      }
      part[tid] = acc;
      __syncthreads();
      if (tid < cc) {
        double t = 0.0;
        for (int q = 0; q < Gc; ++q) t += part[q * cc + tid];
        w[tid] = t;
      }
      __syncthreads();
      for (int64_t e = tid; e < (m - j) * cc; e += 256) {
        const int64_t i = j + e / cc, cl2 = e % cc;
        Q[i * a.ldq + j + c0 + cl2] -= beta * A[i * lda + j] * w[cl2];
      }
      __syncthreads();
    }
  }
}

constexpr int kEigMax = 128;   // largest small factorization done in one workgroup

// ---------------------------------------------------------------------------
// Singular values and left singular vectors of one m x c matrix M (row-major,
// c <= m <= 128) per workgroup: one-sided Jacobi (Hestenes).  Column pairs
// (p, q) in round-robin order are rotated by the c, s that make them
// orthogonal (alpha = |m_p|^2, beta = |m_q|^2, gamma = m_p . m_q,
// zeta = (beta - alpha) / (2 gamma), t = sign(zeta) / (|zeta| +
// sqrt(1 + zeta^2))); a sweep treats every pair once, and sweeps stop when
// every |gamma| <= 1e-15 sqrt(alpha beta), or after 40.  Then M J = U diag(s):
// s_j = |column j|, U's column j = column j / s_j (zero for s_j = 0).  The
// singular values keep an absolute accuracy of about the unit roundoff times
// the largest (no squaring, unlike an eigensolver on M^T M).
// ---------------------------------------------------------------------------
struct SvdArgs {
  const double* M;
  double* U;         // m x c
  double* s;         // c
  int32_t m, c;
};

__global__ void __launch_bounds__(256) jacobi_svd_kernel(const SvdArgs a) {
  extern __shared__ double S[];            // m x (c + 1)
  __shared__ double cs[kEigMax / 2], sn[kEigMax / 2];
  __shared__ int pp[kEigMax / 2], qq[kEigMax / 2];
  __shared__ int pos[kEigMax];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  const int m = a.m, c = a.c, ld = c + 1;
  for (int e = tid; e < m * c; e += 256) S[(e / c) * ld + e % c] = a.M[e];
  const int np = (c + 1) & ~1;
  const int half = np / 2;
  for (int i = tid; i < np; i += 256) pos[i] = i;
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      // four threads per pair form the three dot products
      const int k = tid >> 2, sub = tid & 3;
      double al = 0.0, be = 0.0, ga = 0.0;
      int p = 0, q = -1;
      if (k < half) {
        p = pos[k];
        q = pos[np - 1 - k];
        if (p > q) { const int t = p; p = q; q = t; }
        if (q < c) {
          for (int i = sub; i < m; i += 4) {
            const double x = S[i * ld + p], y = S[i * ld + q];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
        }
      }
      for (int o = 1; o < 4; o <<= 1) {
        al += __shfl_xor(al, o, 64);
        be += __shfl_xor(be, o, 64);
        ga += __shfl_xor(ga, o, 64);
      }
      if (k < half && sub == 0) {
        double cc = 1.0, ss = 0.0;
        if (q < c && ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          cc = 1.0 / sqrt(1.0 + t * t);
          ss = t * cc;
          rotated = 1;
        }
        pp[k] = p;
        qq[k] = (q < c) ? q : -1;
        cs[k] = cc;
        sn[k] = ss;
      }
      __syncthreads();
      for (int e = tid; e < half * m; e += 256) {
        const int k2 = e / m, i = e % m;
        const int q2 = qq[k2];
        if (q2 < 0 || sn[k2] == 0.0) continue;
        const int p2 = pp[k2];
        const double x = S[i * ld + p2], y = S[i * ld + q2];
        S[i * ld + p2] = cs[k2] * x - sn[k2] * y;
        S[i * ld + q2] = sn[k2] * x + cs[k2] * y;
      }
      __syncthreads();
      if (tid == 0) {
        const int last = pos[np - 1];
        for (int i = np - 1; i > 1; --i) pos[i] = pos[i - 1];
        if (np > 1) pos[1] = last;
      }
      __syncthreads();
    }
    if (!rotated) break;
  }
  // column norms and normalised columns
  for (int j = tid; j < c; j += 256) {
    double t = 0.0;
    for (int i = 0; i < m; ++i) t += S[i * ld + j] * S[i * ld + j];
    a.s[j] = sqrt(t);
  }
  __syncthreads();
  for (int e = tid; e < m * c; e += 256) {
    const int i = e / c, j = e % c;
    const double sj = a.s[j];
    a.U[e] = sj > 0.0 ? S[i * ld + j] / sj : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Cores of a QTT matrix product C = A B: C_k[(b, a)][i][j][(b', a')] =
// sum_l A_k[a][i][l][a'] B_k[b][l][j][b'] (A's rank index fastest in each
// merged index).  One thread per output entry.
// ---------------------------------------------------------------------------
struct MatmulCoresArgs {
  const double* A;   // [ra0][m][l][ra1]
  const double* B;   // [rb0][l][n][rb1]
  double* C;         // [rb0 ra0][m][n][rb1 ra1]
  int64_t ra0, ra1, rb0, rb1, m, l, n;
  int64_t total;
};

__global__ void __launch_bounds__(256) matmul_cores_kernel(const MatmulCoresArgs a) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < a.total; e += (int64_t)gridDim.x * 256) {
    int64_t t = e;
    const int64_t ap = t % a.ra1; t /= a.ra1;
    const int64_t bp = t % a.rb1; t /= a.rb1;
    const int64_t j = t % a.n; t /= a.n;
    const int64_t i = t % a.m; t /= a.m;
    const int64_t al = t % a.ra0; t /= a.ra0;
    const int64_t be = t;
    double acc = 0.0;
    for (int64_t q = 0; q < a.l; ++q)
      acc += a.A[((al * a.m + i) * a.l + q) * a.ra1 + ap] * a.B[((be * a.l + q) * a.n + j) * a.rb1 + bp];
    a.C[e] = acc;
  }
}

// ---------------------------------------------------------------------------
// dst[(off0 + a) * n * R1 + i * R1 + off1 + b] += scale * src[(a * n + i) * r1 + b]
// for a < r0, i < n, b < r1: a core added into a block of a larger core
// (blocks of different terms overlap only for a one-core sum).
// ---------------------------------------------------------------------------
struct BlockCopyArgs {
  const double* src;
  double* dst;
  int64_t r0, n, r1;       // source core
  int64_t R1;              // destination's right rank
  int64_t off0, off1;
  double scale;
};

__global__ void __launch_bounds__(256) block_copy_kernel(const BlockCopyArgs a) {
  const int64_t total = a.r0 * a.n * a.r1;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t b = e % a.r1, i = (e / a.r1) % a.n, r = e / (a.r1 * a.n);
    a.dst[((a.off0 + r) * a.n + i) * a.R1 + a.off1 + b] += a.scale * a.src[e];
  }
}

// out[i * r + t] = V[i * ldv + idx[t]] * scale[t]: selected, scaled columns
// (n x r) of a matrix of singular (or eigen) vectors.
struct SelectArgs {
  const double* V;
  const int32_t* idx;
  const double* scale;
  double* out;
  int32_t n, r;
  int32_t ldv;
};

__global__ void __launch_bounds__(256) select_columns_kernel(const SelectArgs a) {
  for (int e = blockIdx.x * 256 + threadIdx.x; e < a.n * a.r; e += gridDim.x * 256) {
    const int i = e / a.r, t = e % a.r;
    a.out[e] = a.V[(int64_t)i * a.ldv + a.idx[t]] * a.scale[t];
  }
}

// row t of M (r x cols) times s[t]
struct ScaleRowsArgs {
  double* M;
  const double* s;
  int64_t r, cols;
};

__global__ void __launch_bounds__(256) scale_rows_kernel(const ScaleRowsArgs a) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < a.r * a.cols; e += (int64_t)gridDim.x * 256)
    a.M[e] *= a.s[e / a.cols];
}

// out[b][i][q] = in[b][q][i] for b < nb, q < nq, i < ni (a batched transpose
// of the last two axes).
struct TransposeArgs {
  const double* in;
  double* out;
  int64_t nb, nq, ni;
};

__global__ void __launch_bounds__(256) transpose_kernel(const TransposeArgs a) {
  const int64_t total = a.nb * a.nq * a.ni;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t q = e % a.nq, i = (e / a.nq) % a.ni, b = e / (a.nq * a.ni);
    a.out[e] = a.in[(b * a.nq + q) * a.ni + i];
  }
}

}  // namespace qtt
