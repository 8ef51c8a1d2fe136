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

// The same rounding in device code on the hardware converter
// (v_cvt_pk_bf16_f32): identical bits to f32_to_bf16_rne for every finite
// value and infinity; a NaN stays a quiet NaN (its payload may differ).
__device__ inline uint16_t bf16_rne_dev(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// FP64 to FP32 rounded to odd: the FP32 value next to x toward zero, with its
// last significand bit set when the conversion is inexact.  FP32 carries 16
// more significand bits than BF16, so rounding this value to BF16 (nearest,
// ties to even) gives the nearest-even BF16 of x itself: one rounding, not
// two (Boldo and Melquiond, "Emulation of FMA and correctly rounded sums:
// proved algorithms using rounding to odd", IEEE Trans. Comput. 57, 2008).
// Infinities, NaNs and exactly representable values pass unchanged; finite
// values beyond the FP32 range become FLT_MAX (odd), which rounds to
// infinity in BF16 as x does.
__device__ __host__ inline float f64_to_f32_odd(double x) {
  const float f = (float)x;
  const double back = (double)f;
  if (back == x || !(x - x == 0.0)) return f;      // exact, or Inf / NaN
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((back < 0 ? -back : back) > (x < 0 ? -x : x)) u -= 1;   // toward zero
  return __builtin_bit_cast(float, u | 1u);
}

__device__ __host__ inline uint16_t f64_to_bf16_rne(double x) { return f32_to_bf16_rne(f64_to_f32_odd(x)); }
__device__ inline uint16_t bf16_rne_dev_f64(double x) { return bf16_rne_dev(f64_to_f32_odd(x)); }

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
  __device__ static elem from_double(double x) { return bf16_rne_dev_f64(x); }
  __device__ static elem from_acc(accel x) { return bf16_rne_dev(x); }
};

// A contiguous run of vectors with its own pointers: used by the first core
// (reads x) and the last core (writes y = z + alpha * (A x), z optional).
// A launch reads its segments from a table in device memory (the head of the
// caller's workspace), sorted by rhs_begin; up to kMaxSeg per launch.
constexpr int kMaxSeg = 4096;
constexpr int kSegChunk = 32;   // segments one table-writing launch carries
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
  int32_t M_bytes;       // bytes of the fragment array M (range of buffer loads), 0 if not needed
  double alpha;
  const Segment* seg;    // device table of nseg segments
};

// Kernel arguments are read in place from the kernarg segment: indexing the
// by-value parameter with a run-time segment number would copy the whole
// struct to scratch memory.
template <class T>
__device__ inline const T& kernarg() {
  return *(const T*)(__builtin_amdgcn_kernarg_segment_ptr());
}

// The segment holding vector rhs: the last one whose rhs_begin <= rhs
// (binary search over the sorted table).
template <class Args>
__device__ inline int find_seg(const Args& a, int64_t rhs) {
  int lo = 0, hi = a.nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.seg[mid].rhs_begin <= rhs) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Copies up to kSegChunk segments carried in the kernel arguments into the
// device table (one launch per chunk; the table then serves every kernel of
// the sweep, and graph capture records these launches with their arguments).
struct SegWriteArgs {
  Segment* dst;
  int32_t n;
  Segment seg[kSegChunk];
};

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

  // Fragment (column block, step) blocks of 64 lanes x E elements.  For
  // BF16, 16 bytes of padding after each 16-lane group move the 16 lanes
  // that store one column's chunk (4 steps x 4 groups, 256 bytes apart
  // unpadded) onto distinct banks; the fragment reads stay contiguous.
  constexpr int PADQ = std::is_same<Tc, bf16_tag>::value ? E : 0;
  constexpr int BLK = 64 * E + 4 * PADQ;
  __shared__ __attribute__((aligned(16))) elem lds[(TC / 16) * SPC * BLK];

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
            lds[(cb * SPC + s) * BLK + (cl + 16 * gq) * E + gq * PADQ + ee] = val;
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
          af[j] = MF::load_frag(&lds[((wc * WC + j) * SPC + s) * BLK + lane * E + (lane >> 4) * PADQ]);
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
// Streamed core step: input in LDS, core fragments straight from L2.
//
// The workgroup walks its (tile, chunk) pairs as one stream.  Input columns
// of a chunk are loaded a chunk ahead into registers, written to one of two
// LDS stages in fragment order, and read by every wave of the workgroup.
// Core fragments never touch LDS: each wave reads the fragments of its own
// row blocks from global memory (they stay L2-resident: one core is at most
// a few hundred KB) one step ahead of the matrix cores, across chunk and
// tile boundaries.  The fragment buffer is padded with zero row blocks up to
// a multiple of 16, so those loads need no bounds test.  One barrier per
// chunk.
// ---------------------------------------------------------------------------
template <class Tc, class Tin, int WAVES_R, int WAVES_C, int WR, int WC, int KC,
          bool ROWS_ON_LANES, bool VEC, int MIN_WAVES = 1>
__global__ void __launch_bounds__(64 * WAVES_R * WAVES_C, MIN_WAVES)
core_step_stream_kernel(const StepArgs args) {
  (void)args;
  const StepArgs& a = kernarg<StepArgs>();
  using MF = Mfma<Tc>;
  using elem = typename MF::elem;
  using frag = typename MF::frag;
  using acc_t = typename MF::acc;
  constexpr int NT = 64 * WAVES_R * WAVES_C;
  constexpr int TC = 16 * WC * WAVES_C;
  constexpr int TR = 16 * WR * WAVES_R;
  constexpr int E = MF::E, KSTEP = MF::KSTEP;
  constexpr int SPC = KC / KSTEP;
  static_assert(KC % KSTEP == 0, "chunk must hold whole steps");
  constexpr int VE = VEC ? (int)(16 / sizeof(Tin)) : 1;
  static_assert(KC % VE == 0, "chunk must hold whole loads");
  constexpr int VPC = KC / VE;
  constexpr int NLA = (TC * VPC + NT - 1) / NT;
  constexpr int A_ELEMS = (TC / 16) * SPC * 64 * E;
  using ld_t = typename std::conditional<VEC, v4u, Tin>::type;

  __shared__ __attribute__((aligned(16))) elem lds[2 * A_ELEMS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave % WAVES_R;
  const int wc = wave / WAVES_R;
  const elem* __restrict__ Mf = reinterpret_cast<const elem*>(a.M);
  const int Ks = a.Ksteps;
  const int nch = (Ks * KSTEP + KC - 1) / KC;

  const int64_t my_tiles = (a.n_tiles > (int64_t)blockIdx.x)
                               ? (a.n_tiles - 1 - (int64_t)blockIdx.x) / gridDim.x + 1 : 0;
  const int64_t total_it = my_tiles * nch;
  if (total_it == 0) return;

  ld_t sa[NLA];
  auto gload = [&](int64_t it) {
    const int64_t tile = blockIdx.x + (it / nch) * (int64_t)gridDim.x;
    const int kc0 = (int)(it % nch) * KC;
    const int64_t col0 = (tile / a.n_row_tiles) * (int64_t)TC;
#pragma unroll
    for (int t = 0; t < NLA; ++t) {
      const int idx = tid + t * NT;
      const int c = idx / VPC;
      const int kap = kc0 + (idx % VPC) * VE;
      const int64_t g = col0 + c;
      sa[t] = ld_t{};
      if (idx < TC * VPC && g < a.ncols && kap < a.K_in) {
        const int64_t rhs = g / a.C;
        const int64_t q = g - rhs * a.C;
        const Tin* p;
        if (a.in_table) {
          const Segment& sg = a.seg[find_seg(a, rhs)];
          p = reinterpret_cast<const Tin*>(sg.x) + (rhs - sg.rhs_begin) * sg.ldx + q * a.K_in;
        } else {
          p = reinterpret_cast<const Tin*>(a.in) + rhs * a.in_stride + q * a.K_in;
        }
        sa[t] = *reinterpret_cast<const ld_t*>(p + kap);
      }
    }
  };
  auto lstore = [&](int stage) {
    elem* A = lds + stage * A_ELEMS;
#pragma unroll
    for (int t = 0; t < NLA; ++t) {
      const int idx = tid + t * NT;
      if (idx < TC * VPC) {
        const int c = idx / VPC;
        const int kl0 = (idx % VPC) * VE;
        const int cb = c >> 4, cl = c & 15;
        const Tin* v = reinterpret_cast<const Tin*>(&sa[t]);
        if constexpr (VE == E && std::is_same<Tin, elem>::value) {
          const int s = kl0 / KSTEP, gq = (kl0 % KSTEP) / E;
          *reinterpret_cast<ld_t*>(&A[((cb * SPC + s) * 64 + cl + 16 * gq) * E]) = sa[t];
        } else {
#pragma unroll
          for (int e = 0; e < VE; ++e) {
            const int kl = kl0 + e;
            const int s = kl / KSTEP, gq = (kl % KSTEP) / E, ee = kl % E;
            elem val;
            if constexpr (std::is_same<Tin, double>::value) val = MF::from_double(v[e]);
            else val = *reinterpret_cast<const elem*>(&v[e]);
            A[((cb * SPC + s) * 64 + cl + 16 * gq) * E + ee] = val;
          }
        }
      }
    }
  };
  // core fragment of row block (this wave's i-th) at global step gs of tile row-tile rt
  auto bload = [&](frag (&dst)[WR], int rt, int gs) {
#pragma unroll
    for (int i = 0; i < WR; ++i) {
      const int rbg = rt * (TR / 16) + wr * WR + i;
      dst[i] = MF::load_frag(Mf + (((int64_t)rbg * Ks + gs) * 64 + lane) * E);
    }
  };

  acc_t acc[WR][WC];
  frag bnext[WR];
  gload(0);
  lstore(0);
  bload(bnext, (int)(((int64_t)blockIdx.x) % a.n_row_tiles), 0);
  __syncthreads();
  if (total_it > 1) gload(1);

  for (int64_t it = 0; it < total_it; ++it) {
    const int ch = (int)(it % nch);
    const int64_t tile = blockIdx.x + (it / nch) * (int64_t)gridDim.x;
    const int rt = (int)(tile % a.n_row_tiles);
    if (ch == 0) {
#pragma unroll
      for (int i = 0; i < WR; ++i)
#pragma unroll
        for (int j = 0; j < WC; ++j) acc[i][j] = acc_t{};
    }
    // where the step after this chunk's last step comes from
    int next_rt = rt, next_s0 = (ch + 1) * SPC;
    if (ch == nch - 1) {
      next_s0 = 0;
      next_rt = (it + 1 < total_it) ? (int)((tile + gridDim.x) % a.n_row_tiles) : rt;
    }
    const elem* A = lds + (it & 1) * A_ELEMS;
    const int s0 = ch * SPC;
    const int nsteps = min(SPC, Ks - s0);
    auto step = [&](int s, bool last) {
      frag bcur[WR];
#pragma unroll
      for (int i = 0; i < WR; ++i) bcur[i] = bnext[i];
      if (!last) bload(bnext, rt, s0 + s + 1);
      else bload(bnext, next_rt, (next_s0 < Ks) ? next_s0 : 0);
      frag af[WC];
#pragma unroll
      for (int j = 0; j < WC; ++j)
        af[j] = MF::load_frag(&A[(((wc * WC + j) * SPC + s) * 64 + lane) * E]);
#pragma unroll
      for (int i = 0; i < WR; ++i)
#pragma unroll
        for (int j = 0; j < WC; ++j)
          acc[i][j] = ROWS_ON_LANES ? MF::mma(af[j], bcur[i], acc[i][j])
                                    : MF::mma(bcur[i], af[j], acc[i][j]);
    };
    if (nsteps == SPC) {
#pragma unroll
      for (int s = 0; s < SPC; ++s) step(s, s == SPC - 1);
    } else {
      for (int s = 0; s < nsteps; ++s) step(s, s == nsteps - 1);
    }

    if (ch == nch - 1) {
      const int64_t col0 = (tile / a.n_row_tiles) * (int64_t)TC;
      const int64_t rhs0 = col0 / a.C;
      const int64_t q0 = col0 - rhs0 * a.C;
      const bool one_rhs = (q0 + TC <= a.C);
      const Segment* s0p = a.out_table ? &a.seg[find_seg(a, rhs0)] : nullptr;
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
    if (it + 1 < total_it) lstore((int)((it + 1) & 1));
    __syncthreads();
    if (it + 2 < total_it) gload(it + 2);
  }
}

// ---------------------------------------------------------------------------
// FP64 core step on the 4x4x4 matrix instruction.
//
// v_mfma_f64_4x4x4_4b_f64 computes four independent 4x4 products over a
// contraction of 4.  Operand lane l carries contraction index l div 16, block
// (l div 4) mod 4 and line l mod 4; output lane 16 r + 4 b + c holds row r,
// column c of block b (measured lane by lane on gfx950).  On gfx950 it runs
// at about twice the FP64 rate of the 16x16x4 form.
//
// Here the four blocks are four groups of four core rows.  The core operand
// is then exactly the 16-row fragment used above (lane 16 k + n holds
// M(16 rb + n, 4 s + k)).  The input operand carries four columns, each
// replicated over the four blocks (lane 16 k + 4 b + c holds b_k(4 s + k,
// column c)), which LDS serves as broadcast reads.  The output of lane l is
// row 16 rb + (l mod 16) of the core, column l div 16 of the 4-column group,
// so rows stay on lanes and 16 lanes store 16 consecutive a_k.
//
// The streaming scheme follows the kernel above: input chunks a chunk ahead
// in registers, two LDS stages; core fragments come from L2 (below).
// LDS input layout: for 4-column group g and step s, a run of 16 values with
// (column c, contraction k) at 4 c + k; runs are kQGS values apart, a padding
// that puts the 16-byte stores of one column's consecutive steps on distinct
// banks.
// ---------------------------------------------------------------------------
static constexpr int kQGS = 20;

// Core fragments come through a buffer resource: the per-lane part of the
// byte offset (row block, lane) is fixed for the whole launch and the step
// part is wave-uniform (a scalar offset), so a fragment load costs no vector
// address arithmetic.  Fragments are prefetched PF steps ahead in a ring of
// registers.  Vector-memory loads complete in issue order, so the wait for a
// fragment also waits for every older load; the next chunk's input loads are
// therefore issued right after the first fragment prefetch of a chunk, which
// leaves them PF + 1 steps before the first wait that covers them.
// Requires Ksteps to be a multiple of the chunk's KC / 4 steps (checked by the
// host): chunks are always whole, so the ring indices stay compile-time.
template <int WAVES_R, int WAVES_C, int WR, int WQ, int KC, int PF, int MIN_WAVES = 1, bool AHEAD = true>
__global__ void __launch_bounds__(64 * WAVES_R * WAVES_C, MIN_WAVES)
core_step_f64q_kernel(const StepArgs args) {
  (void)args;
  const StepArgs& a = kernarg<StepArgs>();
  constexpr int NT = 64 * WAVES_R * WAVES_C;
  constexpr int TC = 4 * WQ * WAVES_C;
  constexpr int TR = 16 * WR * WAVES_R;
  constexpr int SPC = KC / 4;
  static_assert(KC % 8 == 0, "chunk must hold an even number of steps");
  static_assert(SPC % PF == 0, "chunk must hold whole prefetch rounds");
  constexpr int VPC = KC / 2;  // 16-byte loads per column and chunk
  constexpr int NLA = (TC * VPC + NT - 1) / NT;
  constexpr int A_ELEMS = (TC / 4) * SPC * kQGS;

  __shared__ __attribute__((aligned(16))) double lds[2 * A_ELEMS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave % WAVES_R;
  const int wc = wave / WAVES_R;
  const int Ks = a.Ksteps;
  const int nch = (Ks * 4 + KC - 1) / KC;
  // this lane's element inside a 16-value run: column lane mod 4, contraction lane div 16
  const int rd = 4 * (lane & 3) + (lane >> 4);

  const int64_t my_tiles = (a.n_tiles > (int64_t)blockIdx.x)
                               ? (a.n_tiles - 1 - (int64_t)blockIdx.x) / gridDim.x + 1 : 0;
  const int64_t total_it = my_tiles * nch;
  if (total_it == 0) return;

  v4u sa[NLA];
  auto gload = [&](int64_t it) {
    const int64_t tile = blockIdx.x + (it / nch) * (int64_t)gridDim.x;
    const int kc0 = (int)(it % nch) * KC;
    const int64_t col0 = (tile / a.n_row_tiles) * (int64_t)TC;
#pragma unroll
    for (int t = 0; t < NLA; ++t) {
      const int idx = tid + t * NT;
      const int c = idx / VPC;
      const int kap = kc0 + (idx % VPC) * 2;
      const int64_t g = col0 + c;
      sa[t] = v4u{};
      if (idx < TC * VPC && g < a.ncols && kap < a.K_in) {
        const int64_t rhs = g / a.C;
        const int64_t q = g - rhs * a.C;
        const double* p;
        if (a.in_table) {
          const Segment& sg = a.seg[find_seg(a, rhs)];
          p = reinterpret_cast<const double*>(sg.x) + (rhs - sg.rhs_begin) * sg.ldx + q * a.K_in;
        } else {
          p = reinterpret_cast<const double*>(a.in) + rhs * a.in_stride + q * a.K_in;
        }
        sa[t] = *reinterpret_cast<const v4u*>(p + kap);
      }
    }
  };
  auto lstore = [&](int stage) {
    double* A = lds + stage * A_ELEMS;
#pragma unroll
    for (int t = 0; t < NLA; ++t) {
      const int idx = tid + t * NT;
      if (idx < TC * VPC) {
        const int c = idx / VPC;
        const int kl0 = (idx % VPC) * 2;
        *reinterpret_cast<v4u*>(&A[((c >> 2) * SPC + (kl0 >> 2)) * kQGS + 4 * (c & 3) + (kl0 & 3)]) = sa[t];
      }
    }
  };

  // fragment loads: byte offset ((row block) * Ks + step) * 512 + 8 * lane, the
  // row block being rt * TR / 16 + wr * WR + i for row tile rt
  const __amdgpu_buffer_rsrc_t mrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.M), (short)0, a.M_bytes, 0x00020000);
  int vo[WR];
#pragma unroll
  for (int i = 0; i < WR; ++i) vo[i] = ((wr * WR + i) * Ks * 64 + lane) * 8;
  const int rt_bytes = (TR / 16) * Ks * 512;
  // prefetch cursor: step pf_s of the row tile pf_rt (tiles advance by
  // gridDim.x, so the row tile advances by gridDim.x mod n_row_tiles)
  const int rt_adv = (int)(gridDim.x % (unsigned)a.n_row_tiles);
  int pf_s = 0;
  int pf_rt = (int)(blockIdx.x % (unsigned)a.n_row_tiles);
  auto bload = [&](double (&dst)[WR]) {
    const int soff = __builtin_amdgcn_readfirstlane(pf_rt * rt_bytes + pf_s * 512);
#pragma unroll
    for (int i = 0; i < WR; ++i)
      dst[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(mrs, vo[i], soff, 0));
    if (++pf_s == Ks) {
      pf_s = 0;
      pf_rt += rt_adv;
      if (pf_rt >= a.n_row_tiles) pf_rt -= a.n_row_tiles;
    }
  };

  double acc[WR][WQ];
  double ring[PF][WR];
  gload(0);
  lstore(0);
#pragma unroll
  for (int p = 0; p < PF; ++p) bload(ring[p]);
  __syncthreads();

  for (int64_t it = 0; it < total_it; ++it) {
    const int ch = (int)(it % nch);
    const int64_t tile = blockIdx.x + (it / nch) * (int64_t)gridDim.x;
    const int rt = (int)(tile % a.n_row_tiles);
    if (ch == 0) {
#pragma unroll
      for (int i = 0; i < WR; ++i)
#pragma unroll
        for (int j = 0; j < WQ; ++j) acc[i][j] = 0.0;
    }
    const double* A = lds + (it & 1) * A_ELEMS;
    auto lread = [&](double (&dst)[WQ], int s) {
#pragma unroll
      for (int j = 0; j < WQ; ++j) dst[j] = A[((wc * WQ + j) * SPC + s) * kQGS + rd];
    };
    auto mma = [&](const double (&af)[WQ], const double (&bc)[WR]) {
#pragma unroll
      for (int i = 0; i < WR; ++i)
#pragma unroll
        for (int j = 0; j < WQ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[j], bc[i], acc[i][j], 0, 0, 0);
    };
    {
      // ring slot s mod PF holds step s (the ring is back in place after the
      // chunk); with AHEAD, input fragments are read one step ahead (more
      // registers, less exposed LDS latency)
      double af[AHEAD ? 2 : 1][WQ];
      lread(af[0], 0);
#pragma unroll
      for (int s = 0; s < SPC; ++s) {
        if (AHEAD) {
          if (s + 1 < SPC) lread(af[(s + 1) % (AHEAD ? 2 : 1)], s + 1);
        } else if (s > 0) {
          lread(af[0], s);
        }
        double bc[WR];
#pragma unroll
        for (int i = 0; i < WR; ++i) bc[i] = ring[s % PF][i];
        bload(ring[s % PF]);
        if (s == 0 && it + 1 < total_it) gload(it + 1);
        mma(af[AHEAD ? (s & 1) : 0], bc);
      }
    }

    if (ch == nch - 1) {
      const int64_t col0 = (tile / a.n_row_tiles) * (int64_t)TC;
      const int64_t rhs0 = col0 / a.C;
      const int64_t q0 = col0 - rhs0 * a.C;
      const bool one_rhs = (q0 + TC <= a.C);
      const Segment* s0p = a.out_table ? &a.seg[find_seg(a, rhs0)] : nullptr;
#pragma unroll
      for (int i = 0; i < WR; ++i) {
        const int row = rt * TR + (wr * WR + i) * 16 + (lane & 15);
        const int ar = row % a.r_out;
        const int ir = row / a.r_out;
#pragma unroll
        for (int j = 0; j < WQ; ++j) {
          const int cit = (wc * WQ + j) * 4 + (lane >> 4);
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
          const int64_t off = ar + (int64_t)a.r_out * (q + a.C * ir);
          const double val = acc[i][j];
          if (a.out_table) {
            const int64_t vr = rhs - sp->rhs_begin;
            double res = a.alpha * val;
            if (sp->z != nullptr) res += sp->z[vr * sp->ldz + off];
            sp->y[vr * sp->ldy + off] = res;
          } else {
            reinterpret_cast<double*>(a.out)[rhs * a.out_stride + off] = val;
          }
        }
      }
    }
    if (it + 1 < total_it) lstore((int)((it + 1) & 1));
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Two consecutive FP64 core steps k, k + 1 in one pass over a column tile:
// the tile's intermediate y_k stays on chip.
//
// For cores with r_k = RA (24 or 32; with PAD, the RA = 32 kernel takes any
// r_k from 17 to 32, padded) and m_k = n_{k+1} = 8.  A tile is 32
// consecutive columns q = j_{k+1} + 8 Q of b_k, four values of Q.  Step k
// gives phi_k(a_k + RA i_k, j_{k+1} + 8 Q) for all 8 RA rows.  By the row
// separation of step k and the reshape into b_{k+1} (Algorithm 2), these are
// exactly the 32 complete columns q' = Q + (C_k / 8) i_k of b_{k+1}, with
// contraction index a_k + RA j_{k+1}.  They are written to LDS (column
// c' = (Q - Q0) + 4 i_k, all 2 RA steps: 64 KB at RA = 32, so two workgroups
// share a CU), and step k + 1 runs from there with no input traffic and no
// barriers.  Step k streams its input in chunks of KCA / 4 steps through two
// LDS stages that alias the start of the tile, from the packed intermediate
// or, with FIRST, from the caller's FP64 vectors through the segment table
// (core 0); both steps take core fragments through buffer resources with a
// ring of PF prefetched steps.  Step k + 1 covers 64 WRB rows.
//
// Both steps run on v_mfma_f64_16x16x4f64.  One instruction takes 16 tile
// columns (A operand, lane l: column l mod 16, contraction index l div 16)
// against 16 core rows (B operand, lane l: row 16 rb + l mod 16, contraction
// index 4 s + l div 16, the fragment order of the core arrays), so one step
// of a wave is 2 input fragments x WR core fragments -> 2 WR instructions of
// 2048 flops; accumulator lane l, element v holds D(tile column
// (l div 16) + 4 v, core row l mod 16).  Each step reads the next step's
// input fragments from LDS while its own instructions run, and prefetches
// past the end are clamped re-reads instead of branches, so that a whole
// chunk is one block the compiler can schedule across steps.
//
// LDS holds, per 16-column block and step, a 4 x 16 block (contraction
// index, column) whose column is XOR-swizzled with (4 step + contraction
// index) mod 16 (pm_pos): each fragment read is a permutation inside every
// 16-lane group (conflict-free), and the stores of one column's consecutive
// contraction indices fall on distinct banks.
//
// Requirements checked by the host: the conditions above, R_out(k + 1) <=
// 64 WRB, step counts multiples of the chunk (step k) and of 8 (step k + 1),
// C_k % 32 == 0, K_in(k) even with 16-byte aligned columns, both fragment
// arrays below 2 GiB, core k + 1 not the last.
// ---------------------------------------------------------------------------
struct PairArgs {
  const void* MA;        // fragment-ordered FP64 core k (8 RA rows)
  const void* MB;        // fragment-ordered FP64 core k + 1 (K_in = 8 RA)
  const double* in;      // packed b_k (not FIRST)
  double* out;           // packed y_{k+1}
  int64_t in_stride;     // elements between vectors, input
  int64_t out_stride;    // elements between vectors, output
  int64_t C;             // columns of b_k per vector (= columns of b_{k+1})
  int64_t ncols;         // C * nrhs
  int64_t n_tiles;       // ncols / 32
  int32_t KsA, KsB;      // steps of the two cores
  int32_t K_inA;         // r_{k-1} n_k
  int32_t R_outB, r_outB;
  int32_t MA_bytes, MB_bytes;
  int32_t nseg;          // FIRST: input columns come from seg[].x
  int32_t ra;            // boundary rank r_k (the RA = 32 kernels take 17..32)
  const Segment* seg;    // device table of nseg segments
};

// LDS position of (tile column c, contraction index kap) in a tile of
// `steps` steps per 16-column block.
__device__ inline int pm_pos(int c, int kap, int steps) {
  const int s = kap >> 2, k4 = kap & 3;
  return (((c >> 4) * steps + s) * 4 + k4) * 16 + ((c & 15) ^ ((4 * s + k4) & 15));
}

template <int RA, int WRB, bool FIRST, int KCA, int PF, bool PAD = false>
__global__ void __launch_bounds__(256, 2) core_pair_f64_kernel(const PairArgs args) {
  (void)args;
  const PairArgs& a = kernarg<PairArgs>();
  constexpr int NT = 256, TC = 32, CB = TC / 16, SPB = 8;
  constexpr int WRA = RA / 8;                      // 16-row blocks per wave in step k (8 RA rows)
  constexpr int SPA = KCA / 4, VPC = KCA / 2;
  constexpr int PFA = PF < SPA ? PF : SPA;
  constexpr int NLA = (TC * VPC + NT - 1) / NT;
  constexpr int A_ELEMS = CB * SPA * 64;           // one staging stage of step k
  constexpr int KSB = 2 * RA;                      // LDS steps of step k + 1 (K_in <= 8 RA)
  constexpr int X_ELEMS = CB * KSB * 64;           // b_{k+1} tile
  static_assert(RA == 24 || RA == 32, "rank of the fused boundary");
  static_assert(!PAD || RA == 32, "padded ranks use the 256-row kernel");
  static_assert(SPA % PFA == 0 && SPB % PF == 0 && KSB % SPB == 0 && SPB % 4 == 0, "whole prefetch rounds");
  static_assert(2 * A_ELEMS <= X_ELEMS, "stages alias the tile");
  __shared__ __attribute__((aligned(16))) double lds[X_ELEMS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wr = tid >> 6;
  const int k4l = lane >> 4, cl = lane & 15;
  // fragment read offset inside a (column block, step) block, by step mod 4
  int sw[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) sw[t] = 16 * k4l + (cl ^ (4 * t + k4l));
  const int nchA = a.KsA / SPA;
  const int ra = PAD ? a.ra : RA;
  const int kin_b = 8 * ra;
  const int ksb = PAD ? a.KsB : KSB;
  const int64_t my_tiles = (a.n_tiles > (int64_t)blockIdx.x)
                               ? (a.n_tiles - 1 - (int64_t)blockIdx.x) / gridDim.x + 1 : 0;
  if (my_tiles == 0) return;

  v4u sa[NLA];
  auto gload = [&](int64_t tile, int ch) {
    // a tile lies in one vector (C % 32 == 0): its vector, and for FIRST its
    // segment, are wave-uniform (scalar loads)
    const int64_t col0 = tile * TC;
    const int64_t rhs = col0 / a.C;
    const int64_t q0 = col0 - rhs * a.C;
    const double* base;
    if constexpr (FIRST) {
      const Segment& sg = a.seg[find_seg(a, rhs)];
      base = sg.x + (rhs - sg.rhs_begin) * sg.ldx;
    } else {
      base = a.in + rhs * a.in_stride;
    }
    const int kc0 = ch * KCA;
#pragma unroll
    for (int t = 0; t < NLA; ++t) {
      const int idx = tid + t * NT;
      const int c = idx / VPC;
      const int kap = kc0 + (idx % VPC) * 2;
      sa[t] = v4u{};
      // idx is in range by construction when TC * VPC is a multiple of NT,
      // and every column of a tile below n_tiles exists; the contraction
      // index may pass K_in where the core's steps were padded
      const bool inside = ((TC * VPC) % NT == 0 || idx < TC * VPC) && kap < a.K_inA;
      if (inside) sa[t] = *reinterpret_cast<const v4u*>(base + (q0 + c) * a.K_inA + kap);
    }
  };
  auto lstore = [&](int stage) {
    double* S = lds + stage * A_ELEMS;
#pragma unroll
    for (int t = 0; t < NLA; ++t) {
      const int idx = tid + t * NT;
      if (idx < TC * VPC) {
        const int c = idx / VPC;
        const int kl0 = (idx % VPC) * 2;
        typedef double v2d __attribute__((ext_vector_type(2)));
        const v2d v = __builtin_bit_cast(v2d, sa[t]);
        S[pm_pos(c, kl0, SPA)] = v[0];
        S[pm_pos(c, kl0 + 1, SPA)] = v[1];
      }
    }
  };
  const __amdgpu_buffer_rsrc_t rA =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.MA), (short)0, a.MA_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rB =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.MB), (short)0, a.MB_bytes, 0x00020000);
  int voA[WRA], voB[WRB];
#pragma unroll
  for (int i = 0; i < WRA; ++i) voA[i] = ((wr * WRA + i) * a.KsA * 64 + lane) * 8;
#pragma unroll
  for (int i = 0; i < WRB; ++i) voB[i] = ((wr * WRB + i) * a.KsB * 64 + lane) * 8;
  auto loadA = [&](double (&dst)[WRA], int gs) {
    const int soff = __builtin_amdgcn_readfirstlane(gs * 512);
#pragma unroll
    for (int i = 0; i < WRA; ++i)
      dst[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rA, voA[i], soff, 0));
  };
  auto loadB = [&](double (&dst)[WRB], int gs) {
    const int soff = __builtin_amdgcn_readfirstlane(gs * 512);
#pragma unroll
    for (int i = 0; i < WRB; ++i)
      dst[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rB, voB[i], soff, 0));
  };

  // HOLD (the first core's pair, not padded): the first PFA steps of core k
  // (all of them: K_in = 8 is 2 steps) and the first PF steps of core k + 1
  // are the same for every tile; they are loaded once and copied into the
  // rings at the start of each step, so that no step of these short tiles
  // starts by waiting for core fragments.  The padded 256-row kernel would
  // spill, and holding the first steps of core k + 1 in the other pairs
  // measured no gain.
  constexpr bool HOLD = FIRST && !PAD;
  constexpr int HB = HOLD ? PF : 0;
  double holdA[HOLD ? PFA : 1][WRA], holdB[HB > 0 ? HB : 1][WRB];
  if constexpr (HOLD) {
#pragma unroll
    for (int p = 0; p < PFA; ++p) loadA(holdA[p], p);
  }
#pragma unroll
  for (int p = 0; p < HB; ++p) loadB(holdB[p], p);
  // Otherwise the first PFA steps of core k are loaded at the end of the
  // previous tile's step k + 1, before its output stores: loads and stores
  // complete in issue order, so fragments loaded after the stores could not
  // be used before every store had completed.  (Live only across the
  // epilogue, where the ring of core k + 1 is dead; not in the padded
  // kernels, which would spill.)
  constexpr bool NEXTA = !HOLD && !PAD;
  double nextA[NEXTA ? PFA : 1][WRA];
  if constexpr (NEXTA) {
#pragma unroll
    for (int p = 0; p < PFA; ++p) loadA(nextA[p], p);
  }
  gload(blockIdx.x, 0);
  for (int64_t t = 0; t < my_tiles; ++t) {
    const int64_t tile = blockIdx.x + t * (int64_t)gridDim.x;
    // ---- step k: input streamed in chunks of SPA steps ----
    {
      v4d acc[WRA][CB];
      double ring[PFA][WRA];
      __syncthreads();                             // the previous tile's step k + 1 is done with lds
      lstore(0);
#pragma unroll
      for (int p = 0; p < PFA; ++p) {
        if constexpr (HOLD) {
#pragma unroll
          for (int i = 0; i < WRA; ++i) ring[p][i] = holdA[p][i];
        } else if constexpr (NEXTA) {
#pragma unroll
          for (int i = 0; i < WRA; ++i) ring[p][i] = nextA[p][i];
        } else {
          loadA(ring[p], p);
        }
      }
#pragma unroll
      for (int i = 0; i < WRA; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      __syncthreads();
      // Issue priority by phase: the two waves of a SIMD belong to different
      // work-groups, so one is often in another phase of its tile than the
      // other.  The barrier-free step k + 1 outranks step k, and both outrank
      // the output stores and staging at the tile's end, so the matrix pipe
      // is fed first (about 1% on the pairs; the results do not change).
      __builtin_amdgcn_s_setprio(1);
      for (int ch = 0; ch < nchA; ++ch) {
        const double* S = lds + (ch & 1) * A_ELEMS;
        double afn[CB];
#pragma unroll
        for (int j = 0; j < CB; ++j) afn[j] = S[(j * SPA) * 64 + sw[0]];
#pragma unroll
        for (int s = 0; s < SPA; ++s) {
          double af[CB];
#pragma unroll
          for (int j = 0; j < CB; ++j) af[j] = afn[j];
          if (s + 1 < SPA) {
#pragma unroll
            for (int j = 0; j < CB; ++j) afn[j] = S[(j * SPA + s + 1) * 64 + sw[(s + 1) & 3]];
          }
          double bc[WRA];
#pragma unroll
          for (int i = 0; i < WRA; ++i) bc[i] = ring[s % PFA][i];
          const int gs = ch * SPA + s + PFA;
          loadA(ring[s % PFA], gs < a.KsA ? gs : a.KsA - 1);
          if (s == 0) gload(tile, ch + 1 < nchA ? ch + 1 : ch);
#pragma unroll
          for (int i = 0; i < WRA; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[j], bc[i], acc[i][j], 0, 0, 0);
        }
        if (ch + 1 < nchA) {
          lstore((ch + 1) & 1);
          __syncthreads();
        }
      }
      // ---- phi_k tile -> b_{k+1} tile in LDS ----
      __syncthreads();                             // every wave is done with the stages
#pragma unroll
      for (int i = 0; i < WRA; ++i) {
        const int row = 16 * (WRA * wr + i) + cl;            // a_k + ra i_k
        if (row < kin_b) {
          const int ak = row % ra, ik = row / ra;
#pragma unroll
          for (int j = 0; j < CB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int ql = 16 * j + k4l + 4 * v;           // j_{k+1} + 8 (Q - Q0)
              lds[pm_pos((ql >> 3) + 4 * ik, ak + ra * (ql & 7), KSB)] = acc[i][j][v];
            }
        }
      }
      // contraction indices 8 ra .. 4 KsB of every column: zeros
      if (PAD && kin_b < 4 * a.KsB) {
        const int pad = 4 * a.KsB - kin_b;
        for (int e = tid; e < TC * pad; e += NT) {
          const int c = e / pad, kap = kin_b + (e - c * pad);
          lds[pm_pos(c, kap, KSB)] = 0.0;
        }
      }
    }
    // ---- step k + 1 from LDS ----
    v4d acc[WRB][CB];
    double ring[PF][WRB];
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      if (p < HB) {
#pragma unroll
        for (int i = 0; i < WRB; ++i) ring[p][i] = holdB[p][i];
      } else {
        loadB(ring[p], p);
      }
    }
    if (t + 1 < my_tiles) gload(tile + gridDim.x, 0);
#pragma unroll
    for (int i = 0; i < WRB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    __syncthreads();
    __builtin_amdgcn_s_setprio(2);
    double bfn[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) bfn[j] = lds[(j * KSB) * 64 + sw[0]];
    for (int c8 = 0; c8 < ksb / SPB; ++c8) {
#pragma unroll
      for (int s = 0; s < SPB; ++s) {
        const int gs = c8 * SPB + s;
        const int gn = gs + 1 < ksb ? gs + 1 : ksb - 1;
        double af[CB];
#pragma unroll
        for (int j = 0; j < CB; ++j) af[j] = bfn[j];
#pragma unroll
        for (int j = 0; j < CB; ++j) bfn[j] = lds[(j * KSB + gn) * 64 + sw[(s + 1) & 3]];
        double bc[WRB];
#pragma unroll
        for (int i = 0; i < WRB; ++i) bc[i] = ring[s % PF][i];
        loadB(ring[s % PF], gs + PF < ksb ? gs + PF : ksb - 1);
#pragma unroll
        for (int i = 0; i < WRB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[j], bc[i], acc[i][j], 0, 0, 0);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if constexpr (NEXTA) {
      if (t + 1 < my_tiles) {
#pragma unroll
        for (int p = 0; p < PFA; ++p) loadA(nextA[p], p);
      }
    }
    // ---- y_{k+1}(a', q' + C i_{k+1}) with q' = Q + (C / 8) i_k ----
    const int64_t col0 = tile * TC;
    const int64_t rhs = col0 / a.C;
    const int64_t Q0 = (col0 - rhs * a.C) / 8;
    double* dst = a.out + rhs * a.out_stride;
#pragma unroll
    for (int i = 0; i < WRB; ++i) {
      const int row = 16 * (WRB * wr + i) + cl;
      if (row >= a.R_outB) continue;
      const int ar = row % a.r_outB, ir = row / a.r_outB;
#pragma unroll
      for (int j = 0; j < CB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // tile column c' = 16 j + k4l + 4 v = (Q - Q0) + 4 i_k
          const int64_t qp = Q0 + k4l + (a.C / 8) * (4 * j + v);
          dst[ar + (int64_t)a.r_outB * (qp + a.C * ir)] = acc[i][j][v];
        }
    }
  }
}

// ---------------------------------------------------------------------------
// The fused pair of core steps k, k + 1 (see core_pair_f64_kernel) for the
// FP32 sweep, on v_mfma_f32_16x16x4f32 with FP32 accumulation.
//
// Operands as in the streamed FP32 kernels with rows on lanes: the input
// fragment of column block cb and step s has lane l = (column mod 16) +
// 16 (contraction index mod 4); the core fragment lane l holds
// M(16 rb + l mod 16, 4 s + l div 16); accumulator register v of lane l is
// column 4 (l div 16) + v of the 16-column block, core row l mod 16.  A tile
// is 32 columns of b_k (two column blocks); the b_{k+1} tile goes to LDS in
// the same fragment order (column c' = (Q - Q0) + 4 i_k), 32 KB at r_k = 32.
// Requirements as for the FP64 pair.
// ---------------------------------------------------------------------------
template <int RA, int WRB, bool FIRST, int KCA, int PF, bool PAD = false>
__global__ void __launch_bounds__(256, 2) core_pair_f32_kernel(const PairArgs args) {
  (void)args;
  const PairArgs& a = kernarg<PairArgs>();
  using Tin = typename std::conditional<FIRST, double, float>::type;
  constexpr int NT = 256, TC = 32, CB = TC / 16, SPB = 8;
  constexpr int WRA = RA / 8;
  constexpr int SPA = KCA / 4;
  constexpr int VE = 16 / (int)sizeof(Tin);         // values per 16-byte input load
  constexpr int VPC = KCA / VE;
  constexpr int PFA = PF < SPA ? PF : SPA;
  constexpr int NLA = (TC * VPC + NT - 1) / NT;
  constexpr int A_ELEMS = CB * SPA * 64;            // one staging stage of step k
  constexpr int KSB = 2 * RA;                       // LDS steps of step k + 1
  constexpr int X_ELEMS = CB * KSB * 64;            // b_{k+1} tile
  static_assert(RA == 24 || RA == 32, "rank of the fused boundary");
  static_assert(SPA % PFA == 0 && SPB % PF == 0 && KSB % SPB == 0, "whole prefetch rounds");
  static_assert(2 * A_ELEMS <= X_ELEMS, "stages alias the tile");
  __shared__ __attribute__((aligned(16))) float lds[X_ELEMS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wr = tid >> 6;
  const int nchA = a.KsA / SPA;
  static_assert(!PAD || RA == 32, "padded ranks use the 256-row kernel");
  const int ra = PAD ? a.ra : RA;
  const int kin_b = 8 * ra;
  const int ksb = PAD ? a.KsB : KSB;
  const int64_t my_tiles = (a.n_tiles > (int64_t)blockIdx.x)
                               ? (a.n_tiles - 1 - (int64_t)blockIdx.x) / gridDim.x + 1 : 0;
  if (my_tiles == 0) return;

  v4u sa[NLA];
  auto gload = [&](int64_t tile, int ch) {
    const int64_t col0 = tile * TC;
    const int kc0 = ch * KCA;
#pragma unroll
    for (int t = 0; t < NLA; ++t) {
      const int idx = tid + t * NT;
      const int c = idx / VPC;
      const int kap = kc0 + (idx % VPC) * VE;
      const int64_t g = col0 + c;
      sa[t] = v4u{};
      if (idx < TC * VPC && g < a.ncols && kap < a.K_inA) {
        const int64_t rhs = g / a.C;
        const int64_t q = g - rhs * a.C;
        const Tin* p;
        if constexpr (FIRST) {
          const Segment& sg = a.seg[find_seg(a, rhs)];
          p = sg.x + (rhs - sg.rhs_begin) * sg.ldx + q * a.K_inA;
        } else {
          p = reinterpret_cast<const float*>(a.in) + rhs * a.in_stride + q * a.K_inA;
        }
        sa[t] = *reinterpret_cast<const v4u*>(p + kap);
      }
    }
  };
  auto lstore = [&](int stage) {
    float* S = lds + stage * A_ELEMS;
#pragma unroll
    for (int t = 0; t < NLA; ++t) {
      const int idx = tid + t * NT;
      if (idx < TC * VPC) {
        const int c = idx / VPC;
        const int kl0 = (idx % VPC) * VE;
        const Tin* v = reinterpret_cast<const Tin*>(&sa[t]);
#pragma unroll
        for (int e = 0; e < VE; ++e) {
          const int kl = kl0 + e;
          S[((c >> 4) * SPA + (kl >> 2)) * 64 + (c & 15) + 16 * (kl & 3)] = (float)v[e];
        }
      }
    }
  };
  const __amdgpu_buffer_rsrc_t rA =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.MA), (short)0, a.MA_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rB =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.MB), (short)0, a.MB_bytes, 0x00020000);
  int voA[WRA], voB[WRB];
#pragma unroll
  for (int i = 0; i < WRA; ++i) voA[i] = ((wr * WRA + i) * a.KsA * 64 + lane) * 4;
#pragma unroll
  for (int i = 0; i < WRB; ++i) voB[i] = ((wr * WRB + i) * a.KsB * 64 + lane) * 4;
  auto loadA = [&](float (&dst)[WRA], int gs) {
    const int soff = __builtin_amdgcn_readfirstlane(gs * 256);
#pragma unroll
    for (int i = 0; i < WRA; ++i)
      dst[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rA, voA[i], soff, 0));
  };
  auto loadB = [&](float (&dst)[WRB], int gs) {
    const int soff = __builtin_amdgcn_readfirstlane(gs * 256);
#pragma unroll
    for (int i = 0; i < WRB; ++i)
      dst[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rB, voB[i], soff, 0));
  };

  gload(blockIdx.x, 0);
  for (int64_t t = 0; t < my_tiles; ++t) {
    const int64_t tile = blockIdx.x + t * (int64_t)gridDim.x;
    // ---- step k ----
    {
      v4f acc[WRA][CB];
      float ring[PFA][WRA];
      __syncthreads();                             // the previous tile's step k + 1 is done with lds
      lstore(0);
#pragma unroll
      for (int p = 0; p < PFA; ++p) loadA(ring[p], p);
#pragma unroll
      for (int i = 0; i < WRA; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
      __syncthreads();
      for (int ch = 0; ch < nchA; ++ch) {
        const float* S = lds + (ch & 1) * A_ELEMS;
#pragma unroll
        for (int s = 0; s < SPA; ++s) {
          float af[CB];
#pragma unroll
          for (int j = 0; j < CB; ++j) af[j] = S[(j * SPA + s) * 64 + lane];
          float bc[WRA];
#pragma unroll
          for (int i = 0; i < WRA; ++i) bc[i] = ring[s % PFA][i];
          const int gs = ch * SPA + s + PFA;
          if (gs < a.KsA) loadA(ring[s % PFA], gs);
          if (s == 0 && ch + 1 < nchA) gload(tile, ch + 1);
#pragma unroll
          for (int i = 0; i < WRA; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[j], bc[i], acc[i][j], 0, 0, 0);
        }
        if (ch + 1 < nchA) {
          lstore((ch + 1) & 1);
          __syncthreads();
        }
      }
      // ---- phi_k tile -> b_{k+1} tile in LDS ----
      __syncthreads();
#pragma unroll
      for (int i = 0; i < WRA; ++i) {
        const int row = 16 * (WRA * wr + i) + (lane & 15);   // a_k + ra i_k
        if (row < kin_b) {
          const int ak = row % ra, ik = row / ra;
#pragma unroll
          for (int j = 0; j < CB; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int col = 16 * j + 4 * (lane >> 4) + v;  // j_{k+1} + 8 (Q - Q0)
              const int kap = ak + ra * (col & 7);
              const int cp = (col >> 3) + 4 * ik;            // column of b_{k+1} in the tile
              lds[((cp >> 4) * KSB + (kap >> 2)) * 64 + (cp & 15) + 16 * (kap & 3)] = acc[i][j][v];
            }
          }
        }
      }
      if (PAD && kin_b < 4 * a.KsB) {
        const int pad = 4 * a.KsB - kin_b;
        for (int e = tid; e < TC * pad; e += NT) {
          const int c = e / pad, kap = kin_b + (e - c * pad);
          lds[((c >> 4) * KSB + (kap >> 2)) * 64 + (c & 15) + 16 * (kap & 3)] = 0.f;
        }
      }
    }
    // ---- step k + 1 from LDS ----
    v4f acc[WRB][CB];
    float ring[PF][WRB];
#pragma unroll
    for (int p = 0; p < PF; ++p) loadB(ring[p], p);
    if (t + 1 < my_tiles) gload(tile + gridDim.x, 0);
#pragma unroll
    for (int i = 0; i < WRB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
    for (int c8 = 0; c8 < ksb / SPB; ++c8) {
#pragma unroll
      for (int s = 0; s < SPB; ++s) {
        const int gs = c8 * SPB + s;
        float af[CB];
#pragma unroll
        for (int j = 0; j < CB; ++j) af[j] = lds[(j * KSB + gs) * 64 + lane];
        float bc[WRB];
#pragma unroll
        for (int i = 0; i < WRB; ++i) bc[i] = ring[s % PF][i];
        if (gs + PF < ksb) loadB(ring[s % PF], gs + PF);
#pragma unroll
        for (int i = 0; i < WRB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[j], bc[i], acc[i][j], 0, 0, 0);
      }
    }
    // ---- y_{k+1}(a', q' + C i_{k+1}) with q' = Q + (C / 8) i_k ----
    const int64_t col0 = tile * TC;
    const int64_t rhs = col0 / a.C;
    const int64_t Q0 = (col0 - rhs * a.C) / 8;
    float* dst = reinterpret_cast<float*>(a.out) + rhs * a.out_stride;
#pragma unroll
    for (int i = 0; i < WRB; ++i) {
      const int row = 16 * (WRB * wr + i) + (lane & 15);
      if (row >= a.R_outB) continue;
      const int ar = row % a.r_outB, ir = row / a.r_outB;
#pragma unroll
      for (int j = 0; j < CB; ++j) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // column c' = 16 j + 4 (lane div 16) + v = (Q - Q0) + 4 i_k
          const int cp = 16 * j + 4 * (lane >> 4) + v;
          const int64_t qp = Q0 + (cp & 3) + (a.C / 8) * (cp >> 2);
          dst[ar + (int64_t)a.r_outB * (qp + a.C * ir)] = acc[i][j][v];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 core step on the vector ALUs (same intermediate layout as the
// matrix-core kernels, so the two can be mixed core by core).
//
// Lane l owns column q of b_k: its K_in inputs are contiguous, read in groups
// of G consecutive values (G = 8 when K_in % 8 == 0 and columns are 16-byte
// aligned, else 1).  The core values are wave-uniform and come through scalar
// loads as the scalar operand of v_fma_f64 (constant address space).
// Core order: Mv[(g * Rpad + row) * G + e] = M_k(row, G g + e), rows padded to Rpad.
// A workgroup has NW waves; wave w computes rows [row0 + w RW, +RW) of 64 x CPL
// columns (lane l owns columns col0 + l + 64 c).  Output row (a', i) of column
// q goes to a' + r_k (q + C_k i), the row-separating store of Algorithm 2.
// These kernels win on the edge cores (r_0 = 1 or r_d = 1), which are bound
// by memory traffic rather than arithmetic.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(4))) const double cdouble;

struct ValuArgs {
  const double* M;        // Mv (group size G of the kernel)
  const double* in;       // packed input (when in_table == 0)
  double* out;            // packed output (when out_table == 0)
  int64_t in_stride;      // elements between vectors
  int64_t out_stride;
  int64_t C;              // columns per vector
  int64_t ncols;          // C * nrhs
  int64_t n_tiles;        // row tiles * column tiles
  int32_t R_out, Rpad, K_in, r_out;
  int32_t n_row_tiles;
  int32_t in_table, out_table, nseg;
  double alpha;
  const Segment* seg;    // device table of nseg segments
};

// LG > 1: each step loads LG consecutive groups of a column at once (LG G
// values, 128 bytes for G = 8, LG = 2: whole cache lines, so a line is never
// read in halves far apart in time); the FMA chain is unchanged (K_in % (G LG)
// == 0 is checked by the host).
template <int NW, int RW, int CPL, int G, int LG = 1>
__global__ void __launch_bounds__(64 * NW) core_step_valu64_kernel(const ValuArgs args) {
  (void)args;
  const ValuArgs& a = kernarg<ValuArgs>();
  const int lane = threadIdx.x & 63;
  // wave index made provably uniform, so core addresses go through scalar loads
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int TCOL = 64 * CPL;
  const int ngroups = a.K_in / (G * LG);
  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int rt = (int)(tile % a.n_row_tiles);
    const int64_t col0 = (tile / a.n_row_tiles) * TCOL;
    const int row0 = rt * NW * RW + wave * RW;          // wave-uniform
    // x, y and z are device memory: global-address-space pointers, so their
    // accesses are global (vector counter only), not flat instructions that
    // the scalar loads of the core would also wait for
    typedef __attribute__((address_space(1))) double gdouble;
    const gdouble* xin[CPL];
    gdouble* yout[CPL];
    const gdouble* zin[CPL];
    bool ok[CPL];
    const int64_t rhs0 = col0 / a.C;
    if (col0 + TCOL <= (rhs0 + 1) * a.C && col0 + TCOL <= a.ncols) {
      // the whole tile in one vector: its vector and segment are wave-uniform
      const double* xb;
      double* yb;
      const double* zb = nullptr;
      if (a.in_table) {
        const Segment& sg = a.seg[find_seg(a, rhs0)];
        xb = sg.x + (rhs0 - sg.rhs_begin) * sg.ldx;
      } else {
        xb = a.in + rhs0 * a.in_stride;
      }
      if (a.out_table) {
        const Segment& sg = a.seg[find_seg(a, rhs0)];
        yb = sg.y + (rhs0 - sg.rhs_begin) * sg.ldy;
        if (sg.z) zb = sg.z + (rhs0 - sg.rhs_begin) * sg.ldz;
      } else {
        yb = a.out + rhs0 * a.out_stride;
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int64_t q = col0 - rhs0 * a.C + lane + 64 * c;
        ok[c] = true;
        xin[c] = (const gdouble*)(xb + q * a.K_in);
        yout[c] = (gdouble*)(yb + (int64_t)a.r_out * q);
        zin[c] = zb ? (const gdouble*)(zb + (int64_t)a.r_out * q) : nullptr;
      }
    } else {
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int64_t g = col0 + lane + 64 * c;
        ok[c] = g < a.ncols;
        const int64_t gg = ok[c] ? g : 0;
        const int64_t rhs = gg / a.C;
        const int64_t q = gg - rhs * a.C;
        if (a.in_table) {
          const Segment& sg = a.seg[find_seg(a, rhs)];
          xin[c] = (const gdouble*)(sg.x + (rhs - sg.rhs_begin) * sg.ldx + q * a.K_in);
        } else {
          xin[c] = (const gdouble*)(a.in + rhs * a.in_stride + q * a.K_in);
        }
        const int64_t qo = (int64_t)a.r_out * q;
        if (a.out_table) {
          const Segment& sg = a.seg[find_seg(a, rhs)];
          yout[c] = (gdouble*)(sg.y + (rhs - sg.rhs_begin) * sg.ldy + qo);
          zin[c] = sg.z ? (const gdouble*)(sg.z + (rhs - sg.rhs_begin) * sg.ldz + qo) : nullptr;
        } else {
          yout[c] = (gdouble*)(a.out + rhs * a.out_stride + qo);
          zin[c] = nullptr;
        }
      }
    }
    double acc[RW][CPL];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int c = 0; c < CPL; ++c) acc[r][c] = 0.0;

    constexpr int GL = G * LG;
    double x[CPL][GL];
    auto load_x = [&](int gi) {
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const gdouble* p = xin[c] + (int64_t)gi * GL;
#pragma unroll
        for (int e = 0; e < GL; ++e) x[c][e] = p[e];
        if (!ok[c]) {
#pragma unroll
          for (int e = 0; e < GL; ++e) x[c][e] = 0.0;
        }
      }
    };
    load_x(0);
    for (int gi = 0; gi < ngroups; ++gi) {
      double xc[CPL][GL];
#pragma unroll
      for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int e = 0; e < GL; ++e) xc[c][e] = x[c][e];
      if (gi + 1 < ngroups) load_x(gi + 1);
#pragma unroll
      for (int lg = 0; lg < LG; ++lg) {
        const cdouble* mrow = (const cdouble*)a.M + ((int64_t)(gi * LG + lg) * a.Rpad + row0) * G;
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
          for (int e = 0; e < G; ++e) {
            const double mv = mrow[r * G + e];
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc[r][c] = fma(mv, xc[c][lg * G + e], acc[r][c]);
          }
      }
    }
    // every z value of the tile is loaded before any is used, so the loads
    // overlap instead of each waiting for the one before
    double zv[RW][CPL];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int row = min(row0 + r, a.R_out - 1);
      const int ap = row % a.r_out, ir = row / a.r_out;
      const int64_t off = ap + (int64_t)a.r_out * a.C * ir;
#pragma unroll
      for (int c = 0; c < CPL; ++c) zv[r][c] = (a.out_table && ok[c] && zin[c]) ? zin[c][off] : 0.0;
    }
    // results first, then the stores with no load or branch on a lane's
    // data between them (a store never waits for an earlier one)
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        if (a.out_table) {
          double v = a.alpha * acc[r][c];
          if (zin[c]) v += zv[r][c];
          acc[r][c] = v;
        }
      }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int row = row0 + r;
      if (row < a.R_out) {
        const int ap = row % a.r_out, ir = row / a.r_out;
        const int64_t off = ap + (int64_t)a.r_out * a.C * ir;
#pragma unroll
        for (int c = 0; c < CPL; ++c)
          if (ok[c]) yout[c][off] = acc[r][c];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The FP32 last core (R_out = m_d r_d small, packed FP32 input, FP64 output
// z + alpha acc through the segment table) on the vector ALUs.  A wave owns
// RW consecutive rows and 64 CPL consecutive columns of one vector; lane l
// takes columns l + 64 c.  Each output is the FP32 FMA chain over k = 0 ..
// K_in - 1 in order, with core values from the FP32 copy Mv (groups of 8,
// read through the scalar cache: wave-uniform addresses) and the input read
// GL values (GL / 8 groups, whole 128-byte lines for GL = 32) a step ahead.
// Host requirements: last core, K_in % GL == 0, C_d % (64 CPL) == 0,
// 16-byte aligned input.
// ---------------------------------------------------------------------------
template <int RW, int CPL, int GL>
__global__ void __launch_bounds__(64) core_step_valu32_last_kernel(const ValuArgs args) {
  (void)args;
  const ValuArgs& a = kernarg<ValuArgs>();
  const int lane = threadIdx.x & 63;
  constexpr int TCOL = 64 * CPL, G = 8, LG = GL / G;
  typedef __attribute__((address_space(1))) const float gcfloat;
  typedef __attribute__((address_space(1))) double gdouble;
  typedef __attribute__((address_space(1))) const double gcdouble;
  typedef __attribute__((address_space(4))) const float cfloat;
  const int ngroups = a.K_in / GL;
  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int rt = (int)(tile % a.n_row_tiles);
    const int64_t col0 = (tile / a.n_row_tiles) * TCOL;
    const int row0 = rt * RW;
    const int64_t rhs0 = col0 / a.C;                 // the tile lies in one vector
    const Segment& sg = a.seg[find_seg(a, rhs0)];
    gdouble* yb = (gdouble*)(sg.y + (rhs0 - sg.rhs_begin) * sg.ldy);
    gcdouble* zb = sg.z ? (gcdouble*)(sg.z + (rhs0 - sg.rhs_begin) * sg.ldz) : nullptr;
    gcfloat* xb = (gcfloat*)(reinterpret_cast<const float*>(a.in) + rhs0 * a.in_stride);
    int64_t q[CPL];
    gcfloat* xin[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      q[c] = col0 - rhs0 * a.C + lane + 64 * c;
      xin[c] = xb + q[c] * a.K_in;
    }
    float acc[RW][CPL];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int c = 0; c < CPL; ++c) acc[r][c] = 0.f;
    float x[CPL][GL];
    auto load_x = [&](int gi) {
#pragma unroll
      for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int e = 0; e < GL; ++e) x[c][e] = xin[c][(int64_t)gi * GL + e];
    };
    load_x(0);
    for (int gi = 0; gi < ngroups; ++gi) {
      float xc[CPL][GL];
#pragma unroll
      for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int e = 0; e < GL; ++e) xc[c][e] = x[c][e];
      if (gi + 1 < ngroups) load_x(gi + 1);
#pragma unroll
      for (int lg = 0; lg < LG; ++lg) {
        cfloat* mrow = (cfloat*)reinterpret_cast<const float*>(a.M) + ((int64_t)(gi * LG + lg) * a.Rpad + row0) * G;
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
          for (int e = 0; e < G; ++e) {
            const float mv = mrow[r * G + e];
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc[r][c] = fmaf(mv, xc[c][lg * G + e], acc[r][c]);
          }
      }
    }
    // every z value is loaded before any output is formed; the stores then
    // follow with no branch between them when all RW rows exist (a result
    // formed inside a per-row branch would wait there for all earlier stores)
    int64_t off[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int row = min(row0 + r, a.R_out - 1);
      const int ap = row % a.r_out, ir = row / a.r_out;
      off[r] = ap + (int64_t)a.r_out * a.C * ir;
    }
    double res[RW][CPL];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int c = 0; c < CPL; ++c) res[r][c] = zb ? zb[off[r] + (int64_t)a.r_out * q[c]] : 0.0;
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int c = 0; c < CPL; ++c) res[r][c] += a.alpha * (double)acc[r][c];
    if (row0 + RW <= a.R_out) {
#pragma unroll
      for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int c = 0; c < CPL; ++c) yb[off[r] + (int64_t)a.r_out * q[c]] = res[r][c];
    } else {
#pragma unroll
      for (int r = 0; r < RW; ++r)
        if (row0 + r < a.R_out) {
#pragma unroll
          for (int c = 0; c < CPL; ++c) yb[off[r] + (int64_t)a.r_out * q[c]] = res[r][c];
        }
    }
  }
}

// ---------------------------------------------------------------------------
// BF16 interior core step with the core resident in registers.
//
// For the interior cores of the BF16 sweep (R_out = r_k m_k <= 256 and
// K_in = r_{k-1} n_k <= 256, both intermediates packed), the whole core is
// 128 KB: each of the 4 waves keeps the fragments of its 64 rows for every
// contraction step in registers for the life of the workgroup, so the main
// loop moves only the streamed intermediate.  Input tiles of 64 columns are
// contiguous (32 KB at K_in = 256); they are loaded into registers one tile
// ahead and written to one of two LDS stages in fragment order.  The output
// tile is converted to BF16 and written to one of two LDS buffers laid out
// as it lies in memory (for each i_k, the r_k x 64 block a_k + r_k q is
// contiguous), then copied out with 16-byte stores.
// Requirements checked by the host: K_in % 8 == 0, C_k % 64 == 0.
// ---------------------------------------------------------------------------
#ifndef QTT_KERNEL_TEMPLATES_ONLY  // non-template kernels: compiled in the runtime unit only
__global__ void __launch_bounds__(256) core_step_bf16_resident_kernel(const StepArgs args) {
  (void)args;
  const StepArgs& a = kernarg<StepArgs>();
  using MF = Mfma<bf16_tag>;
  constexpr int WR = 4;            // row blocks per wave
  constexpr int TCB = 4;           // column blocks per tile
  constexpr int TC = 16 * TCB;     // 64 columns
  constexpr int KS = 8;            // contraction steps held (K_in <= 256)
  constexpr int NT = 256;
  constexpr int IN_ELEMS = TCB * KS * 64 * 8;      // one input stage (bf16 elements)
  constexpr int OUT_ELEMS = TC * 256;              // one output stage
  constexpr int NSV = (TC * 256 / 8) / NT;         // 16-byte input loads per thread (max)
  __shared__ __attribute__((aligned(16))) uint16_t lin[2 * IN_ELEMS];
  __shared__ __attribute__((aligned(16))) uint16_t lout[2 * OUT_ELEMS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int Ks = a.Ksteps;
  const int vpc = a.K_in / 8;                      // 16-byte vectors per input column
  const int spc = Ks * 4;                          // 16-byte slots per column in LDS (K_in padded)
  const int nslot = TC * spc;                      // per tile
  const uint16_t* __restrict__ Mf = reinterpret_cast<const uint16_t*>(a.M);
  const uint16_t* __restrict__ in = reinterpret_cast<const uint16_t*>(a.in);
  uint16_t* __restrict__ out = reinterpret_cast<uint16_t*>(a.out);

  // resident core fragments
  v8bf mf[WR][KS];
#pragma unroll
  for (int i = 0; i < WR; ++i) {
    const int rbg = wave * WR + i;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      mf[i][s] = MF::zero_frag();
      if (s < Ks && rbg < a.nRB) mf[i][s] = MF::load_frag(Mf + (((int64_t)rbg * Ks + s) * 64 + lane) * 8);
    }
  }

  const int64_t ntiles = a.ncols / TC;
  const int64_t my = (ntiles > (int64_t)blockIdx.x) ? (ntiles - 1 - (int64_t)blockIdx.x) / gridDim.x + 1 : 0;
  if (my == 0) return;

  v4u st[NSV];
  auto gload = [&](int64_t t) {
    const int64_t tile = blockIdx.x + t * (int64_t)gridDim.x;
    const int64_t col0 = tile * TC;
    const v4u* src = reinterpret_cast<const v4u*>(in + col0 * a.K_in);   // packed: tile is contiguous
#pragma unroll
    for (int u = 0; u < NSV; ++u) {
      // slot (c, kv): kv < vpc holds data, kv in [vpc, spc) is the zero padding
      // of the last contraction step (never left stale in LDS)
      const int idx = tid + u * NT;
      const int c = idx / spc;
      const int kv = idx - c * spc;
      st[u] = (idx < nslot && kv < vpc) ? src[c * vpc + kv] : v4u{0u, 0u, 0u, 0u};
    }
  };
  auto lstore = [&](int stage) {
    uint16_t* A = lin + stage * IN_ELEMS;
#pragma unroll
    for (int u = 0; u < NSV; ++u) {
      const int idx = tid + u * NT;
      if (idx < nslot) {
        const int c = idx / spc;
        const int kap = (idx - c * spc) * 8;
        const int s = kap >> 5, g = (kap & 31) >> 3;
        *reinterpret_cast<v4u*>(&A[(((c >> 4) * KS + s) * 64 + (c & 15) + 16 * g) * 8]) = st[u];
      }
    }
  };

  gload(0);
  lstore(0);
  __syncthreads();
  if (my > 1) gload(1);
  const int rows_out = a.R_out;
  const int r = a.r_out;
  for (int64_t t = 0; t < my; ++t) {
    const uint16_t* A = lin + (t & 1) * IN_ELEMS;
    v4f acc[WR][TCB];
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
      for (int j = 0; j < TCB; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      if (s < Ks) {
        v8bf af[TCB];
#pragma unroll
        for (int j = 0; j < TCB; ++j) af[j] = MF::load_frag(&A[((j * KS + s) * 64 + lane) * 8]);
#pragma unroll
        for (int i = 0; i < WR; ++i)
#pragma unroll
          for (int j = 0; j < TCB; ++j) acc[i][j] = MF::mma(mf[i][s], af[j], acc[i][j]);
      }
    }
    // accumulators -> BF16 in the output stage: element (row = a' + r i, col q)
    // sits at i * (r TC) + q r + a'; a lane holds 4 consecutive rows of one column
    uint16_t* O = lout + (t & 1) * OUT_ELEMS;
#pragma unroll
    for (int i = 0; i < WR; ++i) {
      const int row0 = (wave * WR + i) * 16 + 4 * (lane >> 4);
#pragma unroll
      for (int j = 0; j < TCB; ++j) {
        const int q = j * 16 + (lane & 15);
        if ((r & 3) == 0 && row0 + 3 < rows_out) {
          // the 4 rows share i_k and are consecutive a_k: one 8-byte write
          const int ir = row0 / r, ar = row0 - ir * r;
          const uint32_t lo = (uint32_t)MF::from_acc(acc[i][j][0]) | ((uint32_t)MF::from_acc(acc[i][j][1]) << 16);
          const uint32_t hi = (uint32_t)MF::from_acc(acc[i][j][2]) | ((uint32_t)MF::from_acc(acc[i][j][3]) << 16);
          typedef uint32_t v2u __attribute__((ext_vector_type(2)));
          *reinterpret_cast<v2u*>(&O[ir * (r * TC) + q * r + ar]) = v2u{lo, hi};
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = row0 + v;
            if (row < rows_out) {
              const int ir = row / r, ar = row - ir * r;
              O[ir * (r * TC) + q * r + ar] = MF::from_acc(acc[i][j][v]);
            }
          }
        }
      }
    }
    if (t + 1 < my) lstore((int)((t + 1) & 1));
    __syncthreads();
    // copy the output stage out: for each i_k a contiguous run of r * TC values
    {
      const int64_t tile = blockIdx.x + t * (int64_t)gridDim.x;
      const int64_t col0 = tile * TC;
      const int64_t rhs = col0 / a.C;
      const int64_t q0 = col0 - rhs * a.C;
      uint16_t* dst = out + rhs * a.out_stride + (int64_t)r * q0;
      const int m = rows_out / r;
      const int per_i = r * TC / 8;                 // 16-byte vectors per i_k run
      for (int idx = tid; idx < m * per_i; idx += NT) {
        const int ir = idx / per_i;
        const int v = idx - ir * per_i;
        reinterpret_cast<v4u*>(dst + (int64_t)r * a.C * ir)[v] =
            reinterpret_cast<const v4u*>(O + ir * (r * TC))[v];
      }
    }
    if (t + 2 < my) gload(t + 2);
  }
}
#endif  // QTT_KERNEL_TEMPLATES_ONLY

// ---------------------------------------------------------------------------
// Same computation with the input tiles moved by direct global-to-LDS loads
// (tiles of 16 TCB columns: TCB = 4 uses 128 KB of LDS, one workgroup per CU;
// TCB = 2 uses 64 KB, two per CU, so one workgroup's copies and stores
// overlap the other's matrix work)
// (global_load_lds_dwordx4): one instruction fills one 1 KB fragment, lane l
// fetching the 16 bytes of fragment slot l (column l mod 16, contraction
// indices 8 (l div 16) .. +7 of the step).  Three input stages let two tiles
// be in flight while a third is consumed, without staging registers.  Each
// wave waits for its own loads of a tile (vector-memory counter) before the
// barrier that publishes the tile to the other waves.  Slots past K_in (zero
// core values) read the last real indices of the same column, so they hold
// finite data of that column only.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void;

// s_waitcnt with only the vector-memory count limited to N (gfx9 encoding).
template <int N>
__device__ inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (0x7 << 4) | (0xF << 8) | (((N >> 4) & 3) << 14));
}

// s_waitcnt needs an immediate: dispatch a wave-uniform count to one.
template <int I>
__device__ inline void wait_vmcnt_dispatch(int n) {
  if constexpr (I == 0) {
    wait_vmcnt<0>();
  } else {
    if (n >= I) wait_vmcnt<I>();
    else wait_vmcnt_dispatch<I - 1>(n);
  }
}

template <int TCB>
__global__ void __launch_bounds__(256, TCB == 2 ? 2 : 1) core_step_bf16_dma_kernel(const StepArgs args) {
  (void)args;
  const StepArgs& a = kernarg<StepArgs>();
  using MF = Mfma<bf16_tag>;
  constexpr int WR = 4, TC = 16 * TCB, KS = 8, NT = 256;
  constexpr int IN_ELEMS = TCB * KS * 64 * 8;      // 8 KB per column block and stage
  constexpr int OUT_ELEMS = TC * 256;
  constexpr int PER_WAVE = TCB * KS / 4;           // fragment loads per wave per tile (max)
  __shared__ __attribute__((aligned(1024))) uint16_t lin0[IN_ELEMS];
  __shared__ __attribute__((aligned(1024))) uint16_t lin1[IN_ELEMS];
  __shared__ __attribute__((aligned(1024))) uint16_t lin2[IN_ELEMS];
  __shared__ __attribute__((aligned(16))) uint16_t lout[OUT_ELEMS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Ks = a.Ksteps;                         // host guarantees Ks <= KS
  const uint16_t* __restrict__ Mf = reinterpret_cast<const uint16_t*>(a.M);
  const uint16_t* __restrict__ in = reinterpret_cast<const uint16_t*>(a.in);
  uint16_t* __restrict__ out = reinterpret_cast<uint16_t*>(a.out);

  v8bf mf[WR][KS];
#pragma unroll
  for (int i = 0; i < WR; ++i) {
    const int rbg = wave * WR + i;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      mf[i][s] = MF::zero_frag();
      // steps past Ks keep zero core values: their input slots hold clamped data
      if (rbg < a.nRB && s < Ks) mf[i][s] = MF::load_frag(Mf + (((int64_t)rbg * Ks + s) * 64 + lane) * 8);
    }
  }
  wait_vmcnt<0>();
  const int64_t ntiles = a.ncols / TC;
  const int64_t my = (ntiles > (int64_t)blockIdx.x) ? (ntiles - 1 - (int64_t)blockIdx.x) / gridDim.x + 1 : 0;
  if (my == 0) return;

  const int kmax = a.K_in - 8;
  // every wave issues exactly PER_WAVE fragment loads per tile
  auto dma = [&](int64_t t, uint16_t* stage) {
    const int64_t col0 = (blockIdx.x + t * (int64_t)gridDim.x) * TC;
    const uint16_t* base = in + col0 * a.K_in;
#pragma unroll
    for (int u = 0; u < PER_WAVE; ++u) {
      const int f = wave + 4 * u;
      const int cb = f / KS, s = f % KS;
      const int col = cb * 16 + (lane & 15);
      const int kap = min(s * 32 + 8 * (lane >> 4), kmax);
      __builtin_amdgcn_global_load_lds((const void*)(base + (int64_t)col * a.K_in + kap),
                                       (lds_void*)(stage + (cb * KS + s) * 64 * 8), 16, 0, 0);
    }
  };
  auto stage_of = [&](int64_t t) -> uint16_t* {
    const int m3 = (int)(t % 3);
    return m3 == 0 ? lin0 : (m3 == 1 ? lin1 : lin2);
  };

  // Issue order: dma(0..2), then per tile t: [wait for dma(t), barrier,
  // compute, stage output, barrier, stores(t), dma(t+3)].  Vector-memory
  // operations complete in issue order, so dma(t) has landed once at most the
  // operations issued after it are outstanding: dma(t+1), dma(t+2) (those that
  // exist) and the stores of tiles t-2 and t-1.  Every thread issues the same
  // number of stores per tile (R_out TC / 2048; the host requires R_out to be a
  // multiple of 32 for TCB = 4 and of 64 for TCB = 2).  Cores with fewer than
  // KS steps (K_in < 256) copy clamped indices into the unused slots, so the
  // count per wave stays PER_WAVE.
  const int rows_out = a.R_out;
  const int r = a.r_out;
  const int spt = rows_out * TC / (8 * NT);        // 16-byte stores per thread and tile
  // Output staging is swizzled in 16-byte slots: slot v of an i_k run (slots
  // per column spq = r / 8) is stored at v ^ ((column >> 1) & (spq - 1)), so
  // the 8-byte writes of 16 consecutive columns spread over the banks.  Only
  // for spq in {2, 4, 8}; otherwise unswizzled.
  const int spq = r / 8;
  const int swm = (r % 8 == 0 && (spq == 2 || spq == 4 || spq == 8)) ? spq - 1 : 0;
  auto swz = [&](int e, int q) { return ((((e >> 3) ^ ((q >> 1) & swm)) << 3) | (e & 7)); };
  dma(0, lin0);
  if (my > 1) dma(1, lin1);
  if (my > 2) dma(2, lin2);
  for (int64_t t = 0; t < my; ++t) {
    const int nd = (int)(min(my - 1, t + 2) - t);
    const int ns = (int)min(t, (int64_t)2);
    wait_vmcnt_dispatch<2 * PER_WAVE + 16>(nd * PER_WAVE + ns * spt);
    __syncthreads();
    const uint16_t* A = stage_of(t);
    v4f acc[WR][TCB];
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
      for (int j = 0; j < TCB; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      v8bf af[TCB];
#pragma unroll
      for (int j = 0; j < TCB; ++j) af[j] = MF::load_frag(&A[((j * KS + s) * 64 + lane) * 8]);
#pragma unroll
      for (int i = 0; i < WR; ++i)
#pragma unroll
        for (int j = 0; j < TCB; ++j) acc[i][j] = MF::mma(mf[i][s], af[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < WR; ++i) {
      const int row0 = (wave * WR + i) * 16 + 4 * (lane >> 4);
#pragma unroll
      for (int j = 0; j < TCB; ++j) {
        const int q = j * 16 + (lane & 15);
        if ((r & 3) == 0 && row0 + 3 < rows_out) {
          const int ir = row0 / r, ar = row0 - ir * r;
          const uint32_t lo = (uint32_t)MF::from_acc(acc[i][j][0]) | ((uint32_t)MF::from_acc(acc[i][j][1]) << 16);
          const uint32_t hi = (uint32_t)MF::from_acc(acc[i][j][2]) | ((uint32_t)MF::from_acc(acc[i][j][3]) << 16);
          typedef uint32_t v2u __attribute__((ext_vector_type(2)));
          *reinterpret_cast<v2u*>(&lout[ir * (r * TC) + swz(q * r + ar, q)]) = v2u{lo, hi};
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = row0 + v;
            if (row < rows_out) {
              const int ir = row / r, ar = row - ir * r;
              lout[ir * (r * TC) + (swm ? swz(q * r + ar, q) : q * r + ar)] = MF::from_acc(acc[i][j][v]);
            }
          }
        }
      }
    }
    __syncthreads();
    {
      const int64_t col0 = (blockIdx.x + t * (int64_t)gridDim.x) * TC;
      const int64_t rhs = col0 / a.C;
      const int64_t q0 = col0 - rhs * a.C;
      uint16_t* dst = out + rhs * a.out_stride + (int64_t)r * q0;
      const int m = rows_out / r;
      const int per_i = r * TC / 8;
      for (int idx = tid; idx < m * per_i; idx += NT) {
        const int ir = idx / per_i;
        const int v = idx - ir * per_i;
        const int vp = v ^ (((v / (spq > 0 ? spq : 1)) >> 1) & swm);
        reinterpret_cast<v4u*>(dst + (int64_t)r * a.C * ir)[v] =
            reinterpret_cast<const v4u*>(lout + ir * (r * TC))[vp];
      }
    }
    // stage t % 3 was last read by this tile's compute, finished by every
    // wave before the barrier above
    if (t + 3 < my) dma(t + 3, stage_of(t + 3));
    // the stores above read lout; the next tile writes it after the barrier at
    // the top of the loop, which every thread reaches only after its stores
  }
}

// ---------------------------------------------------------------------------
// FP32 interior core step with each product formed on the BF16 matrix
// instruction from a two-term split of both operands.
//
// An FP32 value v is written v_hi + v_lo + e with v_hi = bf16(v) and
// v_lo = bf16(v - v_hi) (nearest even, unit roundoff 2^-8; v - v_hi is exact
// in FP32), so |e| <= 2^-16 |v|.  The product is M b ~ M_hi b_hi + M_hi b_lo
// + M_lo b_hi, accumulated in FP32: the omitted M_lo b_lo and the two
// remainders leave each term's error below about 3 * 2^-16 of its size
// (typically near 2^-19; FP32 products: 2^-24),
// and the three BF16 products cost about a fifth of the FP32 matrix
// instruction's time for the same product (16x16x32 BF16 at 16 times the
// 16x16x4 FP32 rate).  Inputs and outputs stay FP32 in memory.
//
// Workgroup of 8 waves, 32-column tiles; wave w holds the hi and lo core
// fragments of row blocks 2w and 2w + 1 (256 rows) for all 8 steps in
// registers.  A tile's operand buffer in LDS has 16 blocks of 2 KB (column
// block cb, step s: 1 KB of hi fragment, then 1 KB of lo).  Lane l of wave w
// reads, for each of blocks 2w and 2w + 1, the 32 contiguous bytes of its
// fragment slot (column 16 cb + l mod 16, step offsets 8 (l div 16) .. + 7)
// into registers two tiles ahead, splits them and writes its hi and lo
// slots.  Every lane issues the same loads and stores in every tile (tile
// indices past the end are clamped, the stores per lane are the template
// constant SPT = R_out / 64), so the compiler's counter waits stay exact and
// two tiles of loads stay in flight.  Results are staged in LDS laid out as
// in memory (run a + r_k q of r_k TC values per i_k) and leave as 16-byte
// stores.  Host requirements: interior core, K_in <= 256, K_in % 8 == 0,
// R_out = 64 SPT, r_k % 4 == 0, C % 32 == 0, 16-byte aligned input and output.
// ---------------------------------------------------------------------------
__device__ inline uint32_t bf16x2_bits(float a, float b) {
  return (uint32_t)bf16_rne_dev(a) | ((uint32_t)bf16_rne_dev(b) << 16);
}

template <int SPT>
__global__ void __launch_bounds__(512, 2) core_step_f32_split_kernel(const StepArgs args) {
  (void)args;
  const StepArgs& a = kernarg<StepArgs>();
  using MF = Mfma<bf16_tag>;
  constexpr int NW = 8, WR = 2, TCB = 2, TC = 16 * TCB, KS = 8, NT = 64 * NW;
  constexpr int BLK_F = 512;                       // floats per (column block, step) block
  typedef __attribute__((address_space(1))) const v4f gv4f;
  __shared__ __attribute__((aligned(1024))) float lin[TCB * KS * BLK_F];
  __shared__ __attribute__((aligned(16))) float lout[TC * 256];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Ks = a.Ksteps;                         // host guarantees Ks <= KS
  const uint16_t* __restrict__ Mh = reinterpret_cast<const uint16_t*>(a.M);
  const uint16_t* __restrict__ Ml = reinterpret_cast<const uint16_t*>(static_cast<const char*>(a.M) + a.M_bytes);
  float* __restrict__ out = reinterpret_cast<float*>(a.out);

  v8bf mh[WR][KS], ml[WR][KS];
#pragma unroll
  for (int i = 0; i < WR; ++i) {
    const int rbg = wave * WR + i;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      mh[i][s] = MF::zero_frag();
      ml[i][s] = MF::zero_frag();
      if (rbg < a.nRB && s < Ks) {
        const int64_t o = (((int64_t)rbg * Ks + s) * 64 + lane) * 8;
        mh[i][s] = MF::load_frag(Mh + o);
        ml[i][s] = MF::load_frag(Ml + o);
      }
    }
  }
  wait_vmcnt<0>();
  const int64_t ntiles = a.ncols / TC;
  const int64_t my = (ntiles > (int64_t)blockIdx.x) ? (ntiles - 1 - (int64_t)blockIdx.x) / gridDim.x + 1 : 0;
  if (my == 0) return;
  const bool has_rows = wave * WR < a.nRB;

  // this lane's slot in blocks 2w and 2w + 1: column 16 cb + cl, offsets 8 g ..
  const int g = lane >> 4, cl = lane & 15;
  int64_t src[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int blk = 2 * wave + b, cb = blk / KS, s = blk % KS;
    src[b] = (int64_t)(cb * 16 + cl) * a.K_in + min(32 * s + 8 * g, a.K_in - 8);
  }
  gv4f* in = (gv4f*)a.in;
  auto load = [&](int64_t t, v4f (&x)[2][2]) {
    t = min(t, my - 1);                            // clamped: the same loads in every tile
    const int64_t col0 = (blockIdx.x + t * (int64_t)gridDim.x) * TC;
    gv4f* base = (gv4f*)((__attribute__((address_space(1))) const float*)in + col0 * a.K_in);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      gv4f* p = (gv4f*)((__attribute__((address_space(1))) const float*)base + src[b]);
      x[b][0] = p[0];
      x[b][1] = p[1];
    }
  };
  auto split = [&](const v4f (&x)[2][2]) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      float* blk = lin + (2 * wave + b) * BLK_F;
      v4u hi, lo;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const float x0 = x[b][p >> 1][2 * (p & 1)], x1 = x[b][p >> 1][2 * (p & 1) + 1];
        hi[p] = bf16x2_bits(x0, x1);
        lo[p] = bf16x2_bits(x0 - __builtin_bit_cast(float, hi[p] << 16),
                            x1 - __builtin_bit_cast(float, hi[p] & 0xffff0000u));
      }
      *reinterpret_cast<v4u*>(blk + 4 * lane) = hi;
      *reinterpret_cast<v4u*>(blk + 256 + 4 * lane) = lo;
    }
  };

  const int rows_out = a.R_out;                    // = 64 SPT
  const int r = a.r_out;                           // host: r % 4 == 0
  const int spq = r / 4;                           // 16-byte slots per column of one i_k run
  const int swm = (spq == 2 || spq == 4 || spq == 8) ? spq - 1 : 0;
  // one tile: its input (in x) is split into the operand buffer, whose last
  // readers (the previous tile's matrix work) are behind the previous tile's
  // second barrier; x is then refilled with tile t + 2
  auto tile = [&](int64_t t, v4f (&x)[2][2]) {
    split(x);
    load(t + 2, x);
    __syncthreads();
    if (has_rows) {
      v4f acc[WR][TCB];
#pragma unroll
      for (int i = 0; i < WR; ++i)
#pragma unroll
        for (int j = 0; j < TCB; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        if (s < Ks) {
          v8bf ah[TCB], al[TCB];
#pragma unroll
          for (int j = 0; j < TCB; ++j) {
            const float* blk = lin + (j * KS + s) * BLK_F;
            ah[j] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(blk + 4 * lane));
            al[j] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(blk + 256 + 4 * lane));
          }
#pragma unroll
          for (int i = 0; i < WR; ++i)
#pragma unroll
            for (int j = 0; j < TCB; ++j) {
              acc[i][j] = MF::mma(ml[i][s], ah[j], acc[i][j]);
              acc[i][j] = MF::mma(mh[i][s], al[j], acc[i][j]);
              acc[i][j] = MF::mma(mh[i][s], ah[j], acc[i][j]);
            }
        }
      }
#pragma unroll
      for (int i = 0; i < WR; ++i) {
        const int row0 = (wave * WR + i) * 16 + 4 * (lane >> 4);
        if (row0 < rows_out) {                       // rows_out % 64 == 0: all four rows exist
          const int ir = row0 / r, ar = row0 - ir * r;
#pragma unroll
          for (int j = 0; j < TCB; ++j) {
            const int q = j * 16 + (lane & 15);
            const int slot = q * spq + ((ar >> 2) ^ (q & swm));
            *reinterpret_cast<v4f*>(&lout[ir * (r * TC) + 4 * slot]) = acc[i][j];
          }
        }
      }
    }
    __syncthreads();
    const int64_t col0 = (blockIdx.x + t * (int64_t)gridDim.x) * TC;
    const int64_t rhs = col0 / a.C;
    const int64_t q0 = col0 - rhs * a.C;
    float* dst = out + rhs * a.out_stride + (int64_t)r * q0;
    const int per_i = r * TC / 4;
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int idx = tid + u * NT;
      const int ir = idx / per_i;
      const int v = idx - ir * per_i;
      const int q = v / spq, w = v - q * spq;
      const int vp = q * spq + (w ^ (q & swm));
      reinterpret_cast<v4f*>(dst + (int64_t)r * a.C * ir)[v] =
          *reinterpret_cast<const v4f*>(&lout[ir * (r * TC) + 4 * vp]);
    }
    // the next tile writes lout after its first barrier, which every lane
    // reaches only after these reads
  };
  // the first two tiles are peeled so that the loop is entered with the
  // same operations outstanding as on its back edge (the compiler's wait at
  // the loop head serves both)
  v4f xa[2][2], xb[2][2];
  load(0, xa);
  load(1, xb);
  tile(0, xa);
  if (my > 1) {
    tile(1, xb);
    int64_t t = 2;
    for (; t + 1 < my; t += 2) {
      tile(t, xa);
      tile(t + 1, xb);
    }
    if (t < my) tile(t, xa);
  }
}

// ---------------------------------------------------------------------------
// First core step with a short contraction (K_in = n_1 <= 16) on the vector
// ALUs, any compute dtype.
//
// The first core's product is R_out x K_in with K_in = n_1 (8 for octree
// digits): too short a contraction to fill a matrix instruction (the BF16
// one contracts over 32).  The step is bound by writing R_out values per
// column.  Here:
//  * the core, decoded once per workgroup from the dtype's fragment buffer,
//    sits in LDS as Ms[k][row] in the accumulation type (so the values are
//    exactly those the matrix-core kernels use);
//  * a tile of TQ consecutive columns of one vector is read with 16-byte
//    loads into registers a tile ahead, then into LDS (FP64 input, rounded
//    to the compute type as the matrix-core kernels do);
//  * thread t owns column t mod TQ and, in groups of 4 consecutive rows,
//    the rows assigned to its row group; the core rows are LDS broadcasts;
//  * results are staged in LDS laid out as in memory (for each i_1, the run
//    a_1 + r_1 q of r_1 TQ values is contiguous) and leave as 16-byte stores.
// Requirements checked by the host: first core, not the last, K_in <= 16,
// R_out <= 256, r_1 % 4 == 0, C_1 % TQ == 0, FP64 input columns 16-byte
// aligned with an even K_in.
// ---------------------------------------------------------------------------
template <class Tc> struct SmallK;
template <> struct SmallK<double> {
  using acc = double;
  using out = double;
  static constexpr int KS = 4, E = 1, TQ = 8;
  __device__ static acc load_core(const void* M, int64_t i) { return reinterpret_cast<const double*>(M)[i]; }
  __device__ static acc round_in(double x) { return x; }
  __device__ static out to_out(acc v) { return v; }
};
template <> struct SmallK<float> {
  using acc = float;
  using out = float;
  static constexpr int KS = 4, E = 1, TQ = 16;
  __device__ static acc load_core(const void* M, int64_t i) { return reinterpret_cast<const float*>(M)[i]; }
  __device__ static acc round_in(double x) { return (float)x; }
  __device__ static out to_out(acc v) { return v; }
};
template <> struct SmallK<bf16_tag> {
  using acc = float;
  using out = uint16_t;
  static constexpr int KS = 32, E = 8, TQ = 32;
  __device__ static float from_bits(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }
  __device__ static acc load_core(const void* M, int64_t i) { return from_bits(reinterpret_cast<const uint16_t*>(M)[i]); }
  __device__ static acc round_in(double x) { return from_bits(bf16_rne_dev_f64(x)); }
  __device__ static out to_out(acc v) { return bf16_rne_dev(v); }
};

template <class Tc>
__global__ void __launch_bounds__(256) core_step_smallk_kernel(const StepArgs args) {
  (void)args;
  const StepArgs& a = kernarg<StepArgs>();
  using S = SmallK<Tc>;
  using acc_t = typename S::acc;
  using out_t = typename S::out;
  constexpr int NT = 256, TQ = S::TQ, MAXK = 16, MAXR = 256;
  constexpr int RG = NT / TQ;                       // row groups
  constexpr int NLD = (TQ * MAXK / 2 + NT - 1) / NT;  // 16-byte input loads per thread (max)
  __shared__ __attribute__((aligned(16))) acc_t Ms[MAXK * MAXR];
  __shared__ __attribute__((aligned(16))) double xs[TQ * MAXK];
  __shared__ __attribute__((aligned(16))) out_t st[MAXR * TQ];

  const int tid = threadIdx.x;
  const int K = a.K_in, R = a.R_out, r = a.r_out;
  const int Ks = a.Ksteps;
  // core: Ms[k * R + row] = M(row, k), decoded from fragment order
  for (int idx = tid; idx < K * R; idx += NT) {
    const int k = idx / R, row = idx - k * R;
    const int l = (row & 15) + 16 * ((k % S::KS) / S::E);
    Ms[idx] = S::load_core(a.M, (((int64_t)(row >> 4) * Ks + k / S::KS) * 64 + l) * S::E + k % S::E);
  }
  const int64_t ntiles = a.ncols / TQ;
  const int ql = tid % TQ, rg = tid / TQ;
  const int nquad = R / 4;                          // groups of 4 consecutive rows
  const int nvec = TQ * K / 2;
  // the next tile's input is loaded into registers while this tile computes
  v4u pre[NLD];
  auto gload = [&](int64_t tile) {
    const int64_t col0 = tile * TQ;
    const int64_t rhs = col0 / a.C;
    const int64_t q0 = col0 - rhs * a.C;
    const Segment& sg = a.seg[find_seg(a, rhs)];
    const v4u* src = reinterpret_cast<const v4u*>(reinterpret_cast<const double*>(sg.x) +
                                                  (rhs - sg.rhs_begin) * sg.ldx + q0 * K);
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int idx = tid + j * NT;
      if (idx < nvec) pre[j] = src[idx];
    }
  };
  if ((int64_t)blockIdx.x < ntiles) gload(blockIdx.x);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t col0 = tile * TQ;
    const int64_t rhs = col0 / a.C;
    const int64_t q0 = col0 - rhs * a.C;
    __syncthreads();                                // previous tile's xs and staging are free
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int idx = tid + j * NT;
      if (idx < nvec) reinterpret_cast<v4u*>(xs)[idx] = pre[j];
    }
    __syncthreads();
    if (tile + gridDim.x < ntiles) gload(tile + gridDim.x);
    acc_t x[MAXK];
#pragma unroll
    for (int k = 0; k < MAXK; ++k) x[k] = (k < K) ? S::round_in(xs[ql * K + k]) : acc_t(0);
    for (int g = rg; g < nquad; g += RG) {
      const int row0 = 4 * g;
      acc_t v0 = 0, v1 = 0, v2 = 0, v3 = 0;
#pragma unroll
      for (int k = 0; k < MAXK; ++k) {
        if (k < K) {
          const acc_t* m = &Ms[k * R + row0];
          v0 = fma(m[0], x[k], v0);
          v1 = fma(m[1], x[k], v1);
          v2 = fma(m[2], x[k], v2);
          v3 = fma(m[3], x[k], v3);
        }
      }
      // rows row0..row0+3 share i_1 (r_1 % 4 == 0)
      const int ir = row0 / r, ar = row0 - ir * r;
      out_t* o = &st[ir * (r * TQ) + ql * r + ar];
      o[0] = S::to_out(v0);
      o[1] = S::to_out(v1);
      o[2] = S::to_out(v2);
      o[3] = S::to_out(v3);
    }
    __syncthreads();
    // for each i_1 a contiguous run of r TQ values at a_1 + r_1 (q + C_1 i_1)
    out_t* dst = reinterpret_cast<out_t*>(a.out) + rhs * a.out_stride + (int64_t)r * q0;
    const int m = R / r;
    constexpr int VE = 16 / (int)sizeof(out_t);
    const int per_i = r * TQ / VE;
    for (int idx = tid; idx < m * per_i; idx += NT) {
      const int ir = idx / per_i, v = idx - ir * per_i;
      reinterpret_cast<v4u*>(dst + (int64_t)r * a.C * ir)[v] = reinterpret_cast<const v4u*>(st + ir * (r * TQ))[v];
    }
  }
}

// ---------------------------------------------------------------------------
// The last BF16 core (R_out = m_d r_d <= 16) streamed through registers: no
// LDS and no barriers.  Every wave walks its own tiles of 16 columns.  The B
// operand of v_mfma_f32_16x16x32_bf16 (lane l: column l mod 16, contraction
// indices 32 s + 8 (l div 16) .. +7) is loaded straight from the packed
// intermediate, 16 bytes a lane and step, two tiles ahead; the core is held as
// A fragments for every step (rows past R_out are zero).  Accumulator row
// 4 (l div 16) + v, column l mod 16 goes out through the segment table as
// z + alpha acc.  The steps accumulate in order, as in the chunked kernels;
// steps past Ksteps add zero core values times finite data.
// Requirements checked by the host: last core, R_out <= 16, K_in % 8 == 0,
// Ksteps <= KS, C_d % 16 == 0, 16-byte aligned input.
// ---------------------------------------------------------------------------
template <int KS>
__global__ void __launch_bounds__(256) core_step_bf16_last_kernel(const StepArgs args) {
  (void)args;
  const StepArgs& a = kernarg<StepArgs>();
  using MF = Mfma<bf16_tag>;
  const int lane = threadIdx.x & 63;
  // wave index made provably uniform: tile, vector and segment lookups then
  // go through scalar loads, which do not wait on the vector-load counter
  const int64_t gw = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * 4;
  const int Ks = a.Ksteps;
  const uint16_t* __restrict__ Mf = reinterpret_cast<const uint16_t*>(a.M);
  const uint16_t* __restrict__ in = reinterpret_cast<const uint16_t*>(a.in);
  v8bf mf[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
    mf[s] = (s < Ks) ? MF::load_frag(Mf + ((int64_t)s * 64 + lane) * 8) : MF::zero_frag();
  const int64_t ntiles = a.ncols / 16;
  const int cl = lane & 15, kq = 8 * (lane >> 4);
  // indices past K_in (a partial last step) read the column's last 8 values
  // again: finite data of the same column, multiplied by zero core values
  const int kmax = a.K_in - 8;
  // every step is loaded and multiplied (steps past Ks: zero core values
  // times finite data), so the hot loop has no branch on Ks
  auto load = [&](v4u (&b)[KS], int64_t t) {
    const uint16_t* p = in + (t * 16 + cl) * (int64_t)a.K_in;
#pragma unroll
    for (int s = 0; s < KS; ++s) b[s] = *reinterpret_cast<const v4u*>(p + min(32 * s + kq, kmax));
  };
  // A tile's input and z are fetched two tiles ahead (three buffers); vector
  // loads complete in issue order, so a tile's data has arrived once at most
  // the two later fetches and the stores since are outstanding.  The segment
  // of the current vector is cached in scalar registers: a table lookup (a
  // scalar load, which must wait for the wave's earlier stores) happens only
  // when a tile starts a new vector.
  // y and z are device memory: global-address-space pointers, so their
  // accesses are global (vector counter only), not flat instructions
  typedef __attribute__((address_space(1))) double gdouble;
  int64_t cur_rhs = -1;
  gdouble* ybase = nullptr;
  const gdouble* zbase = nullptr;
  auto segment = [&](int64_t rhs) {
    if (rhs != cur_rhs) {
      const Segment& sg = a.seg[find_seg(a, rhs)];
      const int64_t vr = rhs - sg.rhs_begin;
      ybase = (gdouble*)(sg.y + vr * sg.ldy);
      zbase = sg.z ? (const gdouble*)(sg.z + vr * sg.ldz) : nullptr;
      cur_rhs = rhs;
    }
  };
  // one tile in flight: its input steps, z values, output base and z flag
  struct Tile {
    v4u b[KS];
    double z[4];
    gdouble* y;
    bool hz;
  };
  auto fetch = [&](Tile& u, int64_t t) {
    const int64_t col0 = t * 16;
    const int64_t rhs = col0 / a.C;
    const int64_t q = col0 - rhs * a.C + cl;
    segment(rhs);
    u.y = ybase + (int64_t)a.r_out * q;
    u.hz = (zbase != nullptr);
    // the same number of loads on every path (so that the compiler's count
    // of outstanding loads stays exact): without z, the first 8 bytes of the
    // lane's own input column are read and ignored (a cache hit: the column
    // is loaded just after); rows past R_out read row R_out - 1 again
    typedef __attribute__((address_space(1))) const double gcdouble;
    gcdouble* zq = u.hz ? zbase + (int64_t)a.r_out * q : (gcdouble*)(in + (t * 16 + cl) * (int64_t)a.K_in);
    const int64_t zs = u.hz ? (int64_t)a.r_out * a.C : 0;
    const int zr = u.hz ? 1 : 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = min(4 * (lane >> 4) + v, a.R_out - 1);
      const int ir = row / a.r_out, ar = row - ir * a.r_out;
      u.z[v] = zq[zr * ar + zs * ir];
    }
    load(u.b, t);
  };
  auto finish = [&](const Tile& u) {
    v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) acc = MF::mma(mf[s], __builtin_bit_cast(v8bf, u.b[s]), acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * (lane >> 4) + v;
      if (row < a.R_out) {
        const int ir = row / a.r_out, ar = row - ir * a.r_out;
        double res = a.alpha * (double)acc[v];
        if (u.hz) res += u.z[v];
        u.y[ar + (int64_t)a.r_out * a.C * ir] = res;
      }
    }
  };
  if (gw >= ntiles) return;
  const int64_t my = (ntiles - 1 - gw) / nw + 1;   // tiles of this wave: gw + i nw
  auto tile = [&](int64_t i) { return gw + i * nw; };
  Tile u0, u1, u2;
  if (my < 3) {
    fetch(u0, tile(0));
    if (my > 1) fetch(u1, tile(1));
    finish(u0);
    if (my > 1) finish(u1);
    return;
  }
  fetch(u0, tile(0));
  fetch(u1, tile(1));
  int64_t i = 0;
  // steady state, no branch around a vector load: tile i in u0, i + 1 in u1
  for (; i + 4 < my; i += 3) {
    fetch(u2, tile(i + 2));
    finish(u0);
    fetch(u0, tile(i + 3));
    finish(u1);
    fetch(u1, tile(i + 4));
    finish(u2);
  }
  // 2 to 4 tiles left, the first two fetched
  const int64_t left = my - i;
  if (left == 2) {
    finish(u0);
    finish(u1);
  } else if (left == 3) {
    fetch(u2, tile(i + 2));
    finish(u0);
    finish(u1);
    finish(u2);
  } else {
    fetch(u2, tile(i + 2));
    finish(u0);
    fetch(u0, tile(i + 3));
    finish(u1);
    finish(u2);
    finish(u0);
  }
}

// ---------------------------------------------------------------------------
// The first core with K_in <= 8 (r_0 = 1), rows held in registers, for the
// BF16 and FP32 compute types (Tc = bf16_tag, float).
//
// Thread (wave w, lane l): row quad aq = l mod 8 (rows 4 aq .. 4 aq + 3 of an
// i_1 block; active when 4 aq < r_1) and column offset qq = l div 8, for the
// two blocks i_1 = 2 w, 2 w + 1.  A tile is 64 columns; the thread computes
// columns qq + 8 t, t = 0..7, of both blocks.  Each output is the FMA chain
// over k = 0 .. K_in - 1 in order on the BF16-rounded input (the chain of
// core_step_smallk_kernel, so the two agree bitwise).  Its four rows leave as
// one 8-byte (BF16) or 16-byte (FP32) store: with r_1 = 32, the 8 columns x 8
// row quads of a wave are one contiguous run of y_1, and no output passes
// through LDS.  The input is staged in LDS as rounded floats, two buffers
// (one barrier a tile).
// Requirements checked by the host: first core, not the last, K_in <= 8,
// r_1 % 4 == 0, r_1 <= 32, m_1 = R_out / r_1 <= 8, C_1 % 64 == 0, FP64
// input columns 16-byte aligned with an even K_in, output 16-byte aligned.
// ---------------------------------------------------------------------------
template <class Tc, int MAXK>
__global__ void __launch_bounds__(256) core_step_smallk_rows_kernel(const StepArgs args) {
  (void)args;
  const StepArgs& a = kernarg<StepArgs>();
  using S = SmallK<Tc>;
  using out_t = typename S::out;
  constexpr int TQ = 64;
  __shared__ __attribute__((aligned(16))) float xs[2][TQ * MAXK];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int K = a.K_in, r = a.r_out, m = a.R_out / a.r_out;
  const int Ks = a.Ksteps;
  const int aq = lane & 7, qq = lane >> 3;
  const bool act = 4 * aq < r;
  // the core: every load issued unconditionally (indices clamped into the
  // core), then the values outside it replaced by zeros, so that the loads
  // overlap instead of each waiting for the previous one
  float Mr[2][4][MAXK];
#pragma unroll
  for (int ii = 0; ii < 2; ++ii)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int k = 0; k < MAXK; ++k) {
        const int i = 2 * w + ii;
        const int row = min(r * i + 4 * aq + e, a.R_out - 1), kc = min(k, K - 1);
        const int l = (row & 15) + 16 * ((kc % S::KS) / S::E);
        Mr[ii][e][k] = S::load_core(a.M, (((int64_t)(row >> 4) * Ks + kc / S::KS) * 64 + l) * S::E + kc % S::E);
      }
#pragma unroll
  for (int ii = 0; ii < 2; ++ii)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int k = 0; k < MAXK; ++k)
        if (!(act && 2 * w + ii < m && k < K)) Mr[ii][e][k] = 0.f;
  const int64_t ntiles = a.n_tiles;
  const int nvec = TQ * K / 2;                      // 16-byte input loads per tile
  v4u pre = v4u{};
  // with one segment (a single block of vectors) its fields are read once,
  // here, before any barrier: inside the loop a table read could not use the
  // scalar cache and would wait for every outstanding vector access
  const bool one_seg = (a.nseg == 1);
  const double* x0 = a.seg[0].x;
  const int64_t ldx0 = a.seg[0].ldx;
  auto gload = [&](int64_t tile) {
    const int64_t col0 = tile * TQ;
    const int64_t rhs = col0 / a.C;
    const int64_t q0 = col0 - rhs * a.C;
    const double* xv;
    if (one_seg) {
      xv = x0 + rhs * ldx0;
    } else {
      const Segment& sg = a.seg[find_seg(a, rhs)];
      xv = sg.x + (rhs - sg.rhs_begin) * sg.ldx;
    }
    typedef __attribute__((address_space(1))) const v4u gv4u;
    const gv4u* src = (const gv4u*)(xv + q0 * K);
    if (tid < nvec) pre = src[tid];
  };
  if ((int64_t)blockIdx.x < ntiles) gload(blockIdx.x);
  int buf = 0;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x, buf ^= 1) {
    // the buffer was last read two tiles ago, before the previous barrier
    if (tid < nvec) {
      typedef double v2d __attribute__((ext_vector_type(2)));
      const v2d d = __builtin_bit_cast(v2d, pre);
      xs[buf][2 * tid] = S::round_in(d[0]);
      xs[buf][2 * tid + 1] = S::round_in(d[1]);
    }
    __syncthreads();
    if (tile + gridDim.x < ntiles) gload(tile + gridDim.x);
    const int64_t col0 = tile * TQ;
    const int64_t rhs = col0 / a.C;
    const int64_t q0 = col0 - rhs * a.C;
    out_t* dst = reinterpret_cast<out_t*>(a.out) + rhs * a.out_stride + (int64_t)r * q0 + 4 * aq;
    const float* X = xs[buf];
    // fully unrolled: a known number of stores per tile, so the wait before
    // the next tile's staging is counted exactly, not a full drain
#pragma unroll
    for (int t = 0; t < TQ / 8; ++t) {
      const int q = qq + 8 * t;
      float xv[MAXK];
#pragma unroll
      for (int k = 0; k < MAXK; ++k) xv[k] = (k < K) ? X[q * K + k] : 0.f;
#pragma unroll
      for (int ii = 0; ii < 2; ++ii) {
        const int i = 2 * w + ii;
        if (!act || i >= m) continue;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < MAXK; ++k) {
          if (k < K) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = fma(Mr[ii][e][k], xv[k], v[e]);
          }
        }
        if constexpr (sizeof(out_t) == 2) {
          uint2 o;
          o.x = (uint32_t)S::to_out(v[0]) | ((uint32_t)S::to_out(v[1]) << 16);
          o.y = (uint32_t)S::to_out(v[2]) | ((uint32_t)S::to_out(v[3]) << 16);
          *reinterpret_cast<uint2*>(dst + (int64_t)r * (q + a.C * i)) = o;
        } else {
          *reinterpret_cast<v4f*>(dst + (int64_t)r * (q + a.C * i)) = v4f{v[0], v[1], v[2], v[3]};
        }
      }
    }
  }
}

#ifndef QTT_KERNEL_TEMPLATES_ONLY  // non-template kernels: compiled in the runtime unit only
__global__ void __launch_bounds__(64) seg_write_kernel(const SegWriteArgs args) {
  (void)args;
  const SegWriteArgs& a = kernarg<SegWriteArgs>();
  const int t = threadIdx.x;
  if (t < a.n) a.dst[t] = a.seg[t];
}

// ---------------------------------------------------------------------------
// column norms: ||R_c||_2 for every column, two deterministic passes (the
// summation order depends only on the column length, never on the batch).
// ---------------------------------------------------------------------------
constexpr int kNormBlocks = 64;
constexpr int kNormCols = 24;      // columns per norm launch
constexpr int kNormThreads = 256;

struct NormArgs {
  const double* R[kNormCols];
  int64_t ld[kNormCols];
  int64_t col_begin[kNormCols];
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

// ---------------------------------------------------------------------------
// Vector kernels of the flexible GMRES outer solver (section 5.3 uses the
// compressed inverse as the preconditioner of an unrestarted GMRES).  Every
// vector is an FP64 column of N values; column c of basis vector i lies at
// basis + i * bstride + c * N.  The work per call is a few passes over N x K
// FP64 values, so these kernels are HBM-bound: coalesced 8-byte loads, a
// fixed row split and a fixed reduction order (the same result at every
// call, whatever the other columns hold).
// ---------------------------------------------------------------------------

constexpr int kKryCols = 32;       // columns per launch
constexpr int kGramBlocks = 128;   // row chunks per column
constexpr int kGramNb = 16;        // basis vectors per Gram pass (register accumulators)
constexpr int kKryThreads = 256;
constexpr int kKryElems = 4;       // rows per thread per tile

struct GramArgs {
  const double* basis;   // nb basis vectors, stride bstride
  int64_t bstride;
  const double* w;       // w column c at w + c * N
  int64_t N;
  int32_t nb;            // <= kGramNb
  int32_t ncol;          // <= kKryCols
  int32_t col[kKryCols];
  double* partial;       // [(i * ncol + s) * kGramBlocks + block]
};

// partial_i = sum over this block's rows of basis_i * w, for i < nb
__global__ void __launch_bounds__(kKryThreads) gram_partial_kernel(const GramArgs args) {
  (void)args;
  const GramArgs& a = kernarg<GramArgs>();
  const int s = blockIdx.y;
  const int64_t c = a.col[s];
  const int nb = a.nb;
  const int64_t per = (a.N + kGramBlocks - 1) / kGramBlocks;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = min(a.N, b0 + per);
  const double* w = a.w + c * a.N;
  const double* B = a.basis + c * a.N;
  double acc[kGramNb];
#pragma unroll
  for (int i = 0; i < kGramNb; ++i) acc[i] = 0.0;
  constexpr int kTile = kKryThreads * kKryElems;
  for (int64_t t0 = b0; t0 < b1; t0 += kTile) {
    double wv[kKryElems];
#pragma unroll
    for (int e = 0; e < kKryElems; ++e) {
      const int64_t r = t0 + e * kKryThreads + threadIdx.x;
      wv[e] = (r < b1) ? w[r] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kGramNb; ++i) {
      if (i < nb) {
        const double* Bi = B + i * a.bstride;
#pragma unroll
        for (int e = 0; e < kKryElems; ++e) {
          const int64_t r = t0 + e * kKryThreads + threadIdx.x;
          if (r < b1) acc[i] = fma(Bi[r], wv[e], acc[i]);
        }
      }
    }
  }
  // wave sums, then the four waves in order
  __shared__ double red[kKryThreads / 64][kGramNb];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kGramNb; ++i) {
    if (i < nb) {
      double v = acc[i];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) red[wave][i] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nb) {
    const int i = threadIdx.x;
    double v = red[0][i];
#pragma unroll
    for (int q = 1; q < kKryThreads / 64; ++q) v += red[q][i];
    a.partial[((int64_t)i * a.ncol + s) * kGramBlocks + blockIdx.x] = v;
  }
}

// h[(i0 + i) * ncol + s] = sum over blocks (in order) of the partials
__global__ void gram_final_kernel(const double* partial, int nb, int ncol, int i0, double* h) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * ncol) return;
  double v = 0.0;
  for (int b = 0; b < kGramBlocks; ++b) v += partial[(int64_t)t * kGramBlocks + b];
  const int i = t / ncol, s = t - i * ncol;
  h[(int64_t)(i0 + i) * ncol + s] = v;
}

struct CombineArgs {
  double* out;           // column c at out + c * ldo
  int64_t ldo;
  const double* in;      // column c at in + c * ldi; NULL reads as zero
  int64_t ldi;
  const double* scale;   // per slot s (NULL = 1): multiplies in
  const double* basis;   // nb basis vectors, stride bstride, column c at + c * N
  int64_t bstride;
  const double* coef;    // coef[i * ncol + s]
  double sign;           // multiplies the basis sum
  int64_t N;
  int32_t nb;
  int32_t ncol;
  int32_t col[kKryCols];
};

// out = scale_s * in + sign * sum_i coef_is * basis_i  (column by column)
__global__ void __launch_bounds__(kKryThreads) combine_kernel(const CombineArgs args) {
  (void)args;
  const CombineArgs& a = kernarg<CombineArgs>();
  const int s = blockIdx.y;
  const int64_t c = a.col[s];
  const double sc = a.scale ? a.scale[s] : 1.0;
  const double* B = a.basis ? a.basis + c * a.N : nullptr;
  double* out = a.out + c * a.ldo;
  const double* in = a.in ? a.in + c * a.ldi : nullptr;
  const int64_t stride = (int64_t)gridDim.x * kKryThreads;
  for (int64_t r = (int64_t)blockIdx.x * kKryThreads + threadIdx.x; r < a.N; r += stride) {
    double v = 0.0;
    for (int i = 0; i < a.nb; ++i) v = fma(a.coef[(int64_t)i * a.ncol + s], B[i * a.bstride + r], v);
    out[r] = (in ? sc * in[r] : 0.0) + a.sign * v;
  }
}

// y_c += x_c for the columns of one run of consecutive vectors (blockIdx.y
// is the column within the run): the refined solve's sigma += dx when the
// correction dx is kept apart for a residual update.
struct AddColsArgs {
  double* y;
  const double* x;
  int64_t ldy, ldx;      // elements between consecutive columns
  int64_t N;             // rows
};

__global__ void __launch_bounds__(256) add_cols_kernel(const AddColsArgs args) {
  (void)args;
  const AddColsArgs& a = kernarg<AddColsArgs>();
  double* y = a.y + (int64_t)blockIdx.y * a.ldy;
  const double* x = a.x + (int64_t)blockIdx.y * a.ldx;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < a.N; r += stride) y[r] += x[r];
}

// ---------------------------------------------------------------------------
// Non-translation-invariant operators A = a I + B K W C (section 3, the
// matrix form of the Nystrom discretisation): B = diag(b), W C = diag(wc),
// K the QTT matrix.  The diagonals are elementwise passes around K's sweep,
// each one read and one write of the vectors (HBM-bound):
//   before: S[:, t] = wc . x_t            (S dense, column t at S + t * rows)
//   after:  y_t = z_t + alpha (a x_t + b . S[:, t])
// Vector t of the launch belongs to the segment whose rhs_begin is the
// largest one <= t.
// ---------------------------------------------------------------------------

struct DiagArgs {
  const Segment* seg;    // device table of nseg segments
  int32_t nseg;
  int64_t ncol;          // vectors in the launch
  int64_t rows;          // length of the columns handled (N before, M after)
  const double* d;       // wc before, b after; NULL = ones
  double* S;             // scratch, column t at S + t * rows
  double a, alpha;       // after only
};

__device__ inline int diag_segment(const DiagArgs& a, int64_t t) { return find_seg(a, t); }

__global__ void __launch_bounds__(256) diag_in_kernel(const DiagArgs args) {
  (void)args;
  const DiagArgs& a = kernarg<DiagArgs>();
  for (int64_t t = blockIdx.y; t < a.ncol; t += gridDim.y) {
    const Segment& sg = a.seg[diag_segment(a, t)];
    const double* x = sg.x + (t - sg.rhs_begin) * sg.ldx;
    double* out = a.S + t * a.rows;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < a.rows; r += (int64_t)gridDim.x * 256)
      out[r] = a.d ? a.d[r] * x[r] : x[r];
  }
}

__global__ void __launch_bounds__(256) diag_out_kernel(const DiagArgs args) {
  (void)args;
  const DiagArgs& a = kernarg<DiagArgs>();
  for (int64_t t = blockIdx.y; t < a.ncol; t += gridDim.y) {
    const Segment& sg = a.seg[diag_segment(a, t)];
    const int64_t v = t - sg.rhs_begin;
    const double* x = sg.x + v * sg.ldx;
    const double* z = sg.z ? sg.z + v * sg.ldz : nullptr;
    double* y = sg.y + v * sg.ldy;
    const double* T = a.S + t * a.rows;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < a.rows; r += (int64_t)gridDim.x * 256) {
      double u = a.d ? a.d[r] * T[r] : T[r];
      if (a.a != 0.0) u = fma(a.a, x[r], u);
      y[r] = z ? fma(a.alpha, u, z[r]) : a.alpha * u;
    }
  }
}

// ---------------------------------------------------------------------------
// Compressed matrix-vector product (section 4.2): for b in TT form the cores
// of c = A b are
//   c_k[beta][alpha][i][beta'][alpha'] = sum_j G_k[alpha][i][j][alpha'] b_k[beta][j][beta']
// (merged rank index alpha + rA beta).  An output row (v, beta, alpha, i)
// holds R = rA_k rb_k contiguous values; its indices are decoded once per
// row, and the threads run along the row (matrix rank fastest), so the core
// reads of neighbouring lanes are contiguous, the vector-core reads are
// shared and the store is coalesced.  Rows shorter than the block share it.
// The work is n multiply-adds per 8-byte store: HBM-bound on the output.
// ---------------------------------------------------------------------------

struct CmvArgs {
  const double* G;       // [ra0][m][n][ra1]
  const double* B;       // nvec cores [rb0][n][rb1]
  double* C;             // nvec cores [rb0][ra0][m][rb1][ra1]
  int64_t nvec;
  int32_t ra0, ra1, rb0, rb1, m, n;
};

__global__ void __launch_bounds__(256) compressed_matvec_kernel(const CmvArgs args) {
  (void)args;
  const CmvArgs& a = kernarg<CmvArgs>();
  const int R = a.ra1 * a.rb1;
  const int rpb = (R >= 256) ? 1 : 256 / R;                 // rows per block pass
  const int rl = (R >= 256) ? 0 : (int)threadIdx.x / R;      // this thread's row in the pass
  const int q0 = (R >= 256) ? (int)threadIdx.x : (int)threadIdx.x % R;
  const int qs = (R >= 256) ? 256 : R;
  const int64_t rows = a.nvec * a.rb0 * a.ra0 * a.m;
  const int64_t bsz = (int64_t)a.rb0 * a.n * a.rb1;
  if (rl >= rpb) return;
  for (int64_t row0 = (int64_t)blockIdx.x * rpb; row0 < rows; row0 += (int64_t)gridDim.x * rpb) {
    const int64_t row = row0 + rl;
    if (row >= rows) continue;
    int64_t t = row;
    const int i = (int)(t % a.m); t /= a.m;
    const int al = (int)(t % a.ra0); t /= a.ra0;
    const int be = (int)(t % a.rb0); t /= a.rb0;
    const double* g = a.G + ((int64_t)al * a.m + i) * a.n * a.ra1;
    const double* b = a.B + t * bsz + (int64_t)be * a.n * a.rb1;
    double* out = a.C + row * R;
    for (int q = q0; q < R; q += qs) {
      const int ap = q % a.ra1, bp = q / a.ra1;
      double s = 0.0;
      for (int j = 0; j < a.n; ++j) s = fma(g[j * a.ra1 + ap], b[j * a.rb1 + bp], s);
      out[q] = s;
    }
  }
}

// The same product when n <= kCmvMaxN, n rb1 <= kCmvLds and ra1 <= 256 (the
// octree operators): a block takes one vector-core slice b[v][beta] into LDS
// and kCmvRows output rows (alpha, i) of it; a thread keeps the n core
// values G[alpha][i][.][alpha'] in registers and produces the rb1 outputs of
// its alpha' (one global load per output instead of 2n).  Same summation
// order as compressed_matvec_kernel, so the results are identical.
constexpr int kCmvMaxN = 16;
constexpr int kCmvLds = 4096;
constexpr int kCmvRows = 64;

__global__ void __launch_bounds__(256) compressed_matvec_lds_kernel(const CmvArgs args) {
  (void)args;
  const CmvArgs& a = kernarg<CmvArgs>();
  __shared__ double bs[kCmvLds];
  const int n = a.n, ra1 = a.ra1, rb1 = a.rb1;
  const int nrow = a.ra0 * a.m;
  const int nchunk = (nrow + kCmvRows - 1) / kCmvRows;
  const int64_t nblk = a.nvec * a.rb0 * nchunk;
  const int64_t R = (int64_t)ra1 * rb1;
  const int64_t bsz = (int64_t)a.rb0 * n * rb1;
  const int rpp = 256 / ra1;                       // rows in flight per pass
  const int rl = (int)threadIdx.x / ra1, ap = (int)threadIdx.x % ra1;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t vb = blk / nchunk;               // v * rb0 + beta
    const int chunk = (int)(blk - vb * nchunk);
    const int64_t v = vb / a.rb0;
    const int be = (int)(vb - v * a.rb0);
    __syncthreads();                               // the previous slice is no longer read
    const double* b = a.B + v * bsz + (int64_t)be * n * rb1;
    for (int e = threadIdx.x; e < n * rb1; e += 256) bs[e] = b[e];
    __syncthreads();
    if (rl < rpp) {
      const int r1 = min(nrow, (chunk + 1) * kCmvRows);
      for (int r = chunk * kCmvRows + rl; r < r1; r += rpp) {
        const double* g = a.G + (int64_t)r * n * ra1 + ap;   // r = alpha m + i
        double gr[kCmvMaxN];
#pragma unroll
        for (int j = 0; j < kCmvMaxN; ++j) gr[j] = (j < n) ? g[j * ra1] : 0.0;
        double* out = a.C + (vb * nrow + r) * R + ap;
        for (int bp = 0; bp < rb1; ++bp) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < kCmvMaxN; ++j)
            if (j < n) s = fma(gr[j], bs[j * rb1 + bp], s);
          out[(int64_t)bp * ra1] = s;
        }
      }
    }
  }
}

#endif  // QTT_KERNEL_TEMPLATES_ONLY

}  // namespace qtt
