// Device code of libqtt: one core step of the QTT matrix by full-vector
// product (Algorithm 2, section 4.2 of arXiv:1511.06029), as a tiled product
// on the gfx950 matrix cores with the row-separating permutation fused into
// the store.
//
// One core step, for every vector of the batch:
//   b_k   = y_{k-1} viewed as a (r_{k-1} n_k) x C_k matrix (a pure reshape:
//           column q of b_k is K_in = r_{k-1} n_k contiguous values),
//   phi_k = M_k b_k with M_k(a_k + r_k i_k, a_{k-1} + r_{k-1} j_k) = G_k(a_{k-1}, i_k, j_k, a_k),
//   y_k(a_k, q + C_k i_k) = phi_k(a_k + r_k i_k, q)   (the row-separating step),
// so element (row, q) of phi_k is stored at a + r_k (q + C_k i) with
// a = row mod r_k and i = row div r_k.  Several vectors are packed one after
// another, which makes the batch a single product with C_k * nrhs columns.
//
// Matrix-core mapping.  Each 16x16 output block is computed by
// v_mfma_{f64_16x16x4f64, f32_16x16x4f32, f32_16x16x32_bf16}.  An operand
// fragment holds a 16 x KSTEP slice; lane l carries line (l mod 16) and the
// contraction indices KSTEP-slot group (l div 16), E consecutive values each.
// The accumulator of lane l, register v is element (acc_line(l, v), l mod 16)
// of the 16x16 block (first index from operand a, second from operand b), with
// acc_line = 4 (l div 16) + v for the FP32 and BF16 instructions and
// (l div 16) + 4 v for the FP64 one (measured lane by lane on gfx950).
// The same lane mapping is used for the core fragments (stored in this order
// by the loader) and for the input fragments (written in this order into LDS),
// so the contraction index assignment inside a step is immaterial.
//
// ROWS_ON_LANES picks which operand comes first: true puts output rows on the
// 16 lanes of a group (16 consecutive a_k values -> 16 consecutive outputs
// when r_k >= 16), false puts columns there (16 consecutive q -> consecutive
// outputs when r_k = 1, the last core).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtt {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

struct bf16_tag {};  // compute-type tag; elements are stored as uint16_t

__device__ __host__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u) {          // Inf or NaN: keep, quiet the NaN
    return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  }
  u += 0x7fffu + ((u >> 16) & 1u);                 // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}

template <class Tc> struct Mfma;

template <> struct Mfma<double> {
  using elem = double;
  using frag = double;
  using acc = v4d;
  using accel = double;
  static constexpr int E = 1, KSTEP = 4;
  __device__ static acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int acc_line(int lane, int v) { return (lane >> 4) + 4 * v; }
  __device__ static frag load_frag(const elem* p) { return *p; }
  __device__ static frag zero_frag() { return 0.0; }
  __device__ static elem from_double(double x) { return x; }
  __device__ static elem from_acc(accel x) { return x; }
};

template <> struct Mfma<float> {
  using elem = float;
  using frag = float;
  using acc = v4f;
  using accel = float;
  static constexpr int E = 1, KSTEP = 4;
  __device__ static acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int acc_line(int lane, int v) { return 4 * (lane >> 4) + v; }
  __device__ static frag load_frag(const elem* p) { return *p; }
  __device__ static frag zero_frag() { return 0.0f; }
  __device__ static elem from_double(double x) { return (float)x; }
  __device__ static elem from_acc(accel x) { return x; }
};

template <> struct Mfma<bf16_tag> {
  using elem = uint16_t;
  using frag = v8bf;
  using acc = v4f;
  using accel = float;
  static constexpr int E = 8, KSTEP = 32;
  __device__ static acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static int acc_line(int lane, int v) { return 4 * (lane >> 4) + v; }
  __device__ static frag load_frag(const elem* p) {
    return __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(p));
  }
  __device__ static frag zero_frag() { return __builtin_bit_cast(v8bf, v4u{0u, 0u, 0u, 0u}); }
  __device__ static elem from_double(double x) { return f32_to_bf16_rne((float)x); }
  __device__ static elem from_acc(accel x) { return f32_to_bf16_rne(x); }
};

// A contiguous run of vectors with its own pointers: used by the first core
// (reads x) and the last core (writes y = z + alpha * (A x), z optional).
constexpr int kMaxSeg = 24;
struct Segment {
  const double* x;
  double* y;
  const double* z;
  int64_t ldx, ldy, ldz;
  int64_t rhs_begin;  // index of the segment's first vector in the launch
};

struct StepArgs {
  const void* M;         // fragment-ordered core matrix (compute elements)
  const void* in;        // packed input when in_table == 0 (Tin elements)
  void* out;             // packed output when out_table == 0 (compute elements)
  int64_t in_stride;     // elements between vectors, packed input
  int64_t out_stride;    // elements between vectors, packed output
  int64_t C;             // columns of b_k per vector
  int64_t ncols;         // C * nrhs
  int64_t n_tiles;       // n_row_tiles * column tiles
  int32_t R_out;         // r_k m_k
  int32_t K_in;          // r_{k-1} n_k
  int32_t r_out;         // r_k
  int32_t Ksteps;        // ceil(K_in / KSTEP)
  int32_t nRB;           // ceil(R_out / 16)
  int32_t n_row_tiles;
  int32_t in_table;      // input columns come from seg[].x
  int32_t out_table;     // output goes to seg[].y (FP64, with z and alpha)
  int32_t nseg;
  int32_t pad_;
  double alpha;
  Segment seg[kMaxSeg];
};

// Kernel arguments are read in place from the kernarg segment: indexing the
// by-value parameter with a run-time segment number would copy the whole
// struct to scratch memory.
template <class T>
__device__ inline const T& kernarg() {
  return *(const T*)(__builtin_amdgcn_kernarg_segment_ptr());
}

__device__ inline int find_seg(const StepArgs& a, int64_t rhs) {
  int s = 0;
  for (int t = 1; t < a.nseg; ++t) s = (a.seg[t].rhs_begin <= rhs) ? t : s;
  return s;
}

// Tin: element type the input is read in (double for the first core).
// VEC: 16-byte input loads (host guarantees alignment and K_in % (16/sizeof(Tin)) == 0).
template <class Tc, class Tin, int WAVES_R, int WAVES_C, int WR, int WC, int KC,
          bool ROWS_ON_LANES, bool VEC>
__global__ void __launch_bounds__(64 * WAVES_R * WAVES_C)
core_step_kernel(const StepArgs args) {
  (void)args;
  const StepArgs& a = kernarg<StepArgs>();
  using MF = Mfma<Tc>;
  using elem = typename MF::elem;
  using frag = typename MF::frag;
  using acc_t = typename MF::acc;
  constexpr int NT = 64 * WAVES_R * WAVES_C;
  constexpr int TC = 16 * WC * WAVES_C;          // columns per tile
  constexpr int TR = 16 * WR * WAVES_R;          // rows per tile
  constexpr int E = MF::E, KSTEP = MF::KSTEP;
  constexpr int SPC = KC / KSTEP;                // matrix-core steps per chunk
  static_assert(KC % KSTEP == 0, "chunk must hold whole steps");
  constexpr int VE = VEC ? (int)(16 / sizeof(Tin)) : 1;   // input elements per load
  static_assert(KC % VE == 0, "chunk must hold whole loads");
  constexpr int VPC = KC / VE;                   // loads per column per chunk
  constexpr int NLOAD = (TC * VPC + NT - 1) / NT;
  using ld_t = typename std::conditional<VEC, v4u, Tin>::type;

  __shared__ __attribute__((aligned(16))) elem lds[(TC / 16) * SPC * 64 * E];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave % WAVES_R;
  const int wc = wave / WAVES_R;
  const elem* __restrict__ Mf = reinterpret_cast<const elem*>(a.M);
  const int Kpad = a.Ksteps * KSTEP;

  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int rt = (int)(tile % a.n_row_tiles);
    const int64_t col0 = (tile / a.n_row_tiles) * (int64_t)TC;

    // column base pointers of this thread's loads (fixed across chunks)
    const Tin* colp[NLOAD];
    int kofs[NLOAD];
#pragma unroll
    for (int t = 0; t < NLOAD; ++t) {
      const int idx = tid + t * NT;
      const int c = idx / VPC;
      kofs[t] = (idx % VPC) * VE;
      const int64_t g = col0 + c;
      colp[t] = nullptr;
      if (idx < TC * VPC && g < a.ncols) {
        const int64_t rhs = g / a.C;
        const int64_t q = g - rhs * a.C;
        if (a.in_table) {
          const Segment& s = a.seg[find_seg(a, rhs)];
          colp[t] = reinterpret_cast<const Tin*>(s.x) + (rhs - s.rhs_begin) * s.ldx + q * a.K_in;
        } else {
          colp[t] = reinterpret_cast<const Tin*>(a.in) + rhs * a.in_stride + q * a.K_in;
        }
      }
    }

    acc_t acc[WR][WC];
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
      for (int j = 0; j < WC; ++j) acc[i][j] = acc_t{};

    ld_t stage[NLOAD];
    auto load_chunk = [&](int kc0) {
#pragma unroll
      for (int t = 0; t < NLOAD; ++t) {
        const int kap = kc0 + kofs[t];
        if (colp[t] != nullptr && kap < a.K_in) {
          stage[t] = *reinterpret_cast<const ld_t*>(colp[t] + kap);
        } else {
          stage[t] = ld_t{};
        }
      }
    };
    auto store_chunk = [&]() {
#pragma unroll
      for (int t = 0; t < NLOAD; ++t) {
        const int idx = tid + t * NT;
        if (idx < TC * VPC) {
          const int c = idx / VPC;
          const int cb = c >> 4, cl = c & 15;
          const Tin* v = reinterpret_cast<const Tin*>(&stage[t]);
#pragma unroll
          for (int e = 0; e < VE; ++e) {
            const int kl = kofs[t] + e;
            const int s = kl / KSTEP, gq = (kl % KSTEP) / E, ee = kl % E;
            elem val;
            if constexpr (std::is_same<Tin, double>::value) val = MF::from_double(v[e]);
            else val = *reinterpret_cast<const elem*>(&v[e]);
            lds[((cb * SPC + s) * 64 + cl + 16 * gq) * E + ee] = val;
          }
        }
      }
    };

    const int nchunks = (Kpad + KC - 1) / KC;
    load_chunk(0);
    for (int ch = 0; ch < nchunks; ++ch) {
      const int kc0 = ch * KC;
      __syncthreads();                 // previous chunk's fragments consumed
      store_chunk();
      __syncthreads();
      if (ch + 1 < nchunks) load_chunk(kc0 + KC);   // next chunk in flight during compute
      const int s0 = kc0 / KSTEP;
      const int nsteps = min(SPC, a.Ksteps - s0);
      auto step = [&](int s) {
        frag bf[WR];
#pragma unroll
        for (int i = 0; i < WR; ++i) {
          const int rbg = rt * (TR / 16) + wr * WR + i;
          bf[i] = (rbg < a.nRB)
                      ? MF::load_frag(Mf + (((int64_t)rbg * a.Ksteps + s0 + s) * 64 + lane) * E)
                      : MF::zero_frag();
        }
        frag af[WC];
#pragma unroll
        for (int j = 0; j < WC; ++j)
          af[j] = MF::load_frag(&lds[(((wc * WC + j) * SPC + s) * 64 + lane) * E]);
#pragma unroll
        for (int i = 0; i < WR; ++i)
#pragma unroll
          for (int j = 0; j < WC; ++j)
            acc[i][j] = ROWS_ON_LANES ? MF::mma(af[j], bf[i], acc[i][j])
                                      : MF::mma(bf[i], af[j], acc[i][j]);
      };
      if (nsteps == SPC) {
#pragma unroll
        for (int s = 0; s < SPC; ++s) step(s);
      } else {
        for (int s = 0; s < nsteps; ++s) step(s);
      }
    }

    // ---- epilogue: row-separating store (and the fused z + alpha * acc) ----
    const int64_t rhs0 = col0 / a.C;
    const int64_t q0 = col0 - rhs0 * a.C;
    const bool one_rhs = (q0 + TC <= a.C);
    const Segment* s0p = nullptr;
    if (a.out_table) s0p = &a.seg[find_seg(a, rhs0)];
#pragma unroll
    for (int i = 0; i < WR; ++i) {
#pragma unroll
      for (int j = 0; j < WC; ++j) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int row, cit;
          if (ROWS_ON_LANES) {
            cit = (wc * WC + j) * 16 + MF::acc_line(lane, v);
            row = rt * TR + (wr * WR + i) * 16 + (lane & 15);
          } else {
            row = rt * TR + (wr * WR + i) * 16 + MF::acc_line(lane, v);
            cit = (wc * WC + j) * 16 + (lane & 15);
          }
          const int64_t g = col0 + cit;
          if (g >= a.ncols || row >= a.R_out) continue;
          int64_t rhs, q;
          const Segment* sp = s0p;
          if (one_rhs) {
            rhs = rhs0;
            q = q0 + cit;
          } else {
            rhs = g / a.C;
            q = g - rhs * a.C;
            if (a.out_table) sp = &a.seg[find_seg(a, rhs)];
          }
          const int ar = row % a.r_out;
          const int ir = row / a.r_out;
          const int64_t off = ar + (int64_t)a.r_out * (q + a.C * ir);
          const auto val = acc[i][j][v];
          if (a.out_table) {
            const int64_t vr = rhs - sp->rhs_begin;
            double res = a.alpha * (double)val;
            if (sp->z != nullptr) res += sp->z[vr * sp->ldz + off];
            sp->y[vr * sp->ldy + off] = res;
          } else {
            reinterpret_cast<elem*>(a.out)[rhs * a.out_stride + off] = MF::from_acc(val);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// column norms: ||R_c||_2 for every column, two deterministic passes (the
// summation order depends only on the column length, never on the batch).
// ---------------------------------------------------------------------------
constexpr int kNormBlocks = 64;
constexpr int kNormThreads = 256;

struct NormArgs {
  const double* R[kMaxSeg];
  int64_t ld[kMaxSeg];
  int64_t col_begin[kMaxSeg];
  int32_t nseg;
  int32_t ncol;
  int64_t N;
  double* partial;   // ncol * kNormBlocks
};

__global__ void __launch_bounds__(kNormThreads) colnorm_partial_kernel(const NormArgs args) {
  (void)args;
  const NormArgs& a = kernarg<NormArgs>();
  const int c = blockIdx.y;
  int s = 0;
  for (int t = 1; t < a.nseg; ++t) s = (a.col_begin[t] <= c) ? t : s;
  const double* col = a.R[s] + (int64_t)(c - a.col_begin[s]) * a.ld[s];
  const int64_t per = (a.N + kNormBlocks - 1) / kNormBlocks;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = min(a.N, b0 + per);
  double sum = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kNormThreads) {
    const double v = col[i];
    sum = fma(v, v, sum);
  }
  __shared__ double red[kNormThreads];
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int w = kNormThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[(int64_t)c * kNormBlocks + blockIdx.x] = red[0];
}

__global__ void colnorm_final_kernel(const double* partial, int ncol, double* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  double s = 0.0;
  for (int b = 0; b < kNormBlocks; ++b) s += partial[(int64_t)c * kNormBlocks + b];
  out[c] = sqrt(s);
}

}  // namespace qtt
