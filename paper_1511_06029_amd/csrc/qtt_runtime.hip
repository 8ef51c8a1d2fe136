// libqtt host runtime: the C ABI declared in include/qtt.h.
//
// Responsibilities: validate and re-lay out QTT cores into the fragment
// order of the core-step kernels (one device copy per requested dtype),
// drive Algorithm 2 core by core over ping-pong workspace buffers (in waves
// when the workspace is smaller than the batch), pick a kernel configuration
// per core (heuristic or autotuned), run the refined solve, and optionally
// time launches with HIP events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "qtt.h"
#include "qtt_kernels.hpp"
#include "qtt_registry.hpp"
#include "qtt_internal.hpp"

using namespace qtt;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
thread_local std::string g_last_error;

qtt_status_t qtt::fail(qtt_status_t s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

// ---------------------------------------------------------------------------
// dtype helpers
// ---------------------------------------------------------------------------
static int dt_index(qtt_dtype_t t) {
  switch (t) {
    case QTT_FP64: return 0;
    case QTT_FP32: return 1;
    case QTT_BF16: return 2;
  }
  return -1;
}
static const int kKstep[3] = {4, 4, 32};
static const int kElemBytes[3] = {8, 4, 2};
static const int kFragE[3] = {1, 1, 8};

// ---------------------------------------------------------------------------
// kernel registry
// ---------------------------------------------------------------------------
static std::vector<KernelCfg>& registry() {
  static std::vector<KernelCfg> reg = [] {
    std::vector<KernelCfg> v;
    add_kernels_f64(v);
    add_kernels_f32(v);
    add_kernels_bf16(v);
    return v;
  }();
  return reg;
}

static KernelCfg* find_cfg(int dt, bool in_f64, bool vec, int id) {
  for (auto& k : registry())
    if (k.dt == dt && k.in_f64 == in_f64 && k.vec == vec && k.id == id) return &k;
  return nullptr;
}

// Row blocks to allocate for a core with nRB real ones: the largest
// ceil(nRB / t) * t over the tile heights t (in row blocks) of the registry.
static int padded_row_blocks(int nRB) {
  int pad = nRB;
  for (auto& k : registry()) {
    const int t = k.TR / 16;
    pad = std::max(pad, (nRB + t - 1) / t * t);
  }
  return pad;
}

// Shape ids available for (dtype, input type) with vector loads.
static std::vector<int> shape_ids(int dt, bool in_f64) {
  std::vector<int> ids;
  for (auto& k : registry())
    if (k.dt == dt && k.in_f64 == in_f64 && k.vec) ids.push_back(k.id);
  return ids;
}

static std::vector<ValuCfg>& valu_registry() {
  static std::vector<ValuCfg> reg = [] {
    std::vector<ValuCfg> v;
    add_valu_kernels(v);
    return v;
  }();
  return reg;
}

static ValuCfg* find_valu(int id) {
  for (auto& k : valu_registry())
    if (k.id == id) return &k;
  return nullptr;
}

// Rows of the FP64 vector-ALU core copy: every tile height divides it.
static int valu_padded_rows(int R_out) {
  int pad = R_out;
  for (auto& k : valu_registry()) {
    const int t = k.NW * k.RW;
    pad = std::max(pad, (R_out + t - 1) / t * t);
  }
  return pad;
}

// BF16 interior kernel with the core resident in registers (shape id 30).
static const int kBf16Resident = 30;
static KernelCfg* bf16_resident_cfg() {
  static KernelCfg k = [] {
    KernelCfg c;
    c.dt = 2;
    c.in_f64 = false;
    c.vec = true;
    c.TR = 256;
    c.TC = 64;
    c.KC = 256;
    c.NT = 256;
    c.id = kBf16Resident;
    c.fn = reinterpret_cast<const void*>(&core_step_bf16_resident_kernel);
    c.occ = 0;
    c.kind = -1;
    return c;
  }();
  return &k;
}

// BF16 interior kernel fed by direct global-to-LDS loads: 64-column tiles
// (shape id 31, one workgroup per CU) or 32-column tiles (id 33, two).
static const int kBf16Dma = 31;
static const int kBf16Dma32 = 33;
static KernelCfg* bf16_dma_cfg() {
  static KernelCfg k = [] {
    KernelCfg c = *bf16_resident_cfg();
    c.id = kBf16Dma;
    c.fn = bf16_dma_kernel(4);
    c.occ = 0;
    c.kind = -1;
    return c;
  }();
  return &k;
}
// The last BF16 core streamed through registers (shape id 35).
static const int kBf16Last = 35;
static KernelCfg* bf16_last_cfg() {
  static KernelCfg k = [] {
    KernelCfg c = *bf16_resident_cfg();
    c.id = kBf16Last;
    c.TR = 16;
    c.TC = 16;
    c.KC = 256;
    c.fn = bf16_last_kernel();
    c.occ = 0;
    c.kind = -1;
    return c;
  }();
  return &k;
}
static KernelCfg* bf16_dma32_cfg() {
  static KernelCfg k = [] {
    KernelCfg c = *bf16_resident_cfg();
    c.id = kBf16Dma32;
    c.TC = 32;
    c.fn = bf16_dma_kernel(2);
    c.occ = 0;
    c.kind = -1;
    return c;
  }();
  return &k;
}

// FP32 interior cores with the products formed from split BF16 operands
// (shape id 38, core_step_f32_split_kernel): never chosen by the heuristic
// or the autotuner (its rounding error is up to about 3 * 2^-16 per product
// term against 2^-24), only
// when pinned with qtt_set_shape.  One instantiation per R_out / 64.
static const int kF32Split = 38;
// FP32 last core on the vector ALUs (the FP32 default for R_out <= 16)
static const int kValu32 = 39;
static KernelCfg* f32_split_cfg(int spt) {
  static KernelCfg k[4] = {};
  static std::once_flag once;
  std::call_once(once, [] {
    for (int i = 0; i < 4; ++i) {
      k[i].dt = 1;
      k[i].in_f64 = false;
      k[i].vec = true;
      k[i].TR = 256;
      k[i].TC = 32;
      k[i].KC = 256;
      k[i].NT = 512;
      k[i].id = kF32Split;
      k[i].fn = f32_split_kernel(i + 1);
      k[i].occ = 0;
      k[i].kind = -1;
    }
  });
  return &k[spt - 1];
}

// First core with a short contraction on the vector ALUs (shape id 34), one
// instantiation per compute dtype.
static KernelCfg* smallk_cfg(int dt) {
  static KernelCfg k[3] = {};
  static std::once_flag once;
  std::call_once(once, [] {
    const void* fns[3] = {smallk_kernel(0), smallk_kernel(1), smallk_kernel(2)};
    const int tq[3] = {SmallK<double>::TQ, SmallK<float>::TQ, SmallK<bf16_tag>::TQ};
    for (int t = 0; t < 3; ++t) {
      k[t].dt = t;
      k[t].in_f64 = true;
      k[t].vec = true;
      k[t].TR = 256;
      k[t].TC = tq[t];
      k[t].KC = 16;
      k[t].NT = 256;
      k[t].id = kSmallK;
      k[t].fn = fns[t];
      k[t].occ = 0;
      k[t].kind = -1;
    }
  });
  return &k[dt];
}

// The BF16 and FP32 first cores with rows in registers
// (core_step_smallk_rows_kernel): also configuration 34, 64-column tiles.
static KernelCfg* smallk_rows_cfg(int dt) {
  static KernelCfg k[2] = {};
  static std::once_flag once;
  std::call_once(once, [] {
    for (int i = 0; i < 2; ++i) {
      k[i].dt = i == 0 ? 2 : 1;
      k[i].in_f64 = true;
      k[i].vec = true;
      k[i].TR = 256;
      k[i].TC = 64;
      k[i].KC = 8;
      k[i].NT = 256;
      k[i].id = kSmallK;
      k[i].fn = smallk_kernel(i == 0 ? 3 : 4);
      k[i].occ = 0;
      k[i].kind = -1;
    }
  });
  return &k[dt == 2 ? 0 : 1];
}

static int num_cus() {
  static int n = [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return cus > 0 ? cus : 256;
  }();
  return n;
}

static std::mutex g_occ_mu;
static int occupancy_fn(const void* fn, int nt, int* cache) {
  std::lock_guard<std::mutex> lk(g_occ_mu);
  if (*cache == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, nt, 0) != hipSuccess || nb < 1) nb = 1;
    *cache = nb;
  }
  return *cache;
}
static int occupancy(KernelCfg* k) {
  std::lock_guard<std::mutex> lk(g_occ_mu);
  if (k->occ == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k->fn, k->NT, 0) != hipSuccess || nb < 1) nb = 1;
    k->occ = nb;
  }
  return k->occ;
}

// ---------------------------------------------------------------------------
// the handle's graph cache
// ---------------------------------------------------------------------------
static const size_t kMaxGraphs = 48;

// Destroys a cached graph once its last launch (on whatever stream) is done.
static void destroy_graph(const qtt_matrix_s::Graph& g) {
  if (g.done) {
    (void)hipEventSynchronize(g.done);
    (void)hipEventDestroy(g.done);
  }
  (void)hipGraphExecDestroy(g.exec);
  (void)hipGraphDestroy(g.graph);
}

static void drop_graphs(const qtt_matrix_s* A) {
  std::lock_guard<std::mutex> lk(A->graph_mu);
  for (auto& g : A->graphs) destroy_graph(g);
  A->graphs.clear();
  ++A->tune_gen;
}

static bool valid_handle(qtt_matrix_t A) { return A != nullptr && A->d > 0; }

// Process-wide table of tuned shapes, keyed by (dtype, R_out, K_in, r_out, C).
// It does not depend on the number of vectors, so a vector's kernels (and
// hence its bits) are the same whatever batch it is part of.
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int, int64_t>, int> g_tuned;
// bumped on every change of g_tuned: part of every graph key, so that no
// handle replays a sweep captured with configurations that changed since
static std::atomic<int64_t> g_tune_gen{0};

static bool tune_log() {
  const char* s = getenv("QTT_TUNE_LOG");
  return s && s[0] == '1';
}

// Untuned defaults, from tuning runs on MI355X at L = 7, r = 32.
static int heuristic_shape(int R_out, int K_in, int dt) {
  if (R_out <= 16) return dt == 0 ? 49 : (dt == 2 ? kBf16Last : kValu32);   // last core (r_d = 1; 49
                                                 // needs K_in % 16 == 0, else 47; 35 and 39 fall back to 2)
  if (dt == 0 && R_out > 64) {                   // FP64: 4x4x4 matrix instruction
    if (K_in <= 16) return 67;                   // short chunks for the first core
    return R_out <= 192 ? 63 : 75;
  }
  if (K_in <= 16) return dt == 0 ? 6 : kSmallK; // first core (r_0 = 1; falls back to 26)
  if (R_out <= 64) return kGenericShape;
  return dt == 2 ? kBf16Dma32 : 21;              // interior cores (falls back to 31, then resident)
}

// ---------------------------------------------------------------------------
// timing
// ---------------------------------------------------------------------------
struct TimedLaunch {
  hipEvent_t a, b;
  int dt, pos;
  int shape;  // kernel configuration id
  double flops, bytes;
};
static thread_local bool g_timing = false;
static thread_local std::vector<TimedLaunch> g_timed;
static std::atomic<int> g_timing_env{-1};

static thread_local bool g_timing_off = false;   // set while an entry point must not create events

static bool timing_on() {
  if (g_timing_off) return false;
  if (g_timing) return true;
  int e = g_timing_env.load();
  if (e < 0) {
    const char* s = getenv("QTT_TIMING");
    e = (s && s[0] == '1') ? 1 : 0;
    g_timing_env.store(e);
  }
  return e == 1;
}

// ---------------------------------------------------------------------------
// launching one core step
// ---------------------------------------------------------------------------
// FP64 vector-ALU shape ids are 40..49; anything else is a matrix-core shape.
static bool is_valu_shape(int id) { return id >= 40 && id < 50; }
// The FP32 last core on the vector ALUs (core_step_valu32_kernel, id kValu32).
static ValuCfg* valu32_cfg() {
  static ValuCfg k = valu32_last_cfg();
  return &k;
}

static void record_timing(TimedLaunch& tl, const qtt_matrix_s* A, int k, int dt, int64_t ncols,
                          const Segment* segs, int nseg, int shape);

// dt 0: the FP64 vector-ALU configurations (id 40..49); dt 1: the FP32 last
// core (kValu32; the caller checks its requirements).
static qtt_status_t launch_valu(const qtt_matrix_s* A, int k, int dt, int64_t nrhs, const Segment* segs, int nseg,
                                const Segment* dsegs, const void* in_packed, void* out_packed, double alpha, int id,
                                hipStream_t st) {
  const CoreDev& c = A->core[k];
  const bool first = (k == 0), last = (k == A->d - 1);
  ValuCfg* vc = (dt == 1) ? valu32_cfg() : find_valu(id);
  // grouped kernels read each lane's inputs as aligned 16-byte vectors
  bool aligned = (c.K_in % 8) == 0 && c.valu != nullptr;
  if (first) {
    for (int s = 0; s < nseg && aligned; ++s)
      aligned = (reinterpret_cast<uintptr_t>(segs[s].x) % 16 == 0) && (segs[s].ldx % 2 == 0);
  } else {
    aligned = aligned && (reinterpret_cast<uintptr_t>(in_packed) % 16 == 0);
  }
  if (dt == 0 && vc && c.K_in % (vc->G * vc->LG) != 0) vc = find_valu(47);
  if (dt == 0 && (!vc || (vc->G == 8 && !aligned))) vc = find_valu(kValuGeneric);
  ValuArgs a;
  memset(&a, 0, sizeof(a));
  a.M = (dt == 1) ? reinterpret_cast<const double*>(c.valu32) : (vc->G == 8) ? c.valu : c.valu1;
  a.in = static_cast<const double*>(in_packed);
  a.out = static_cast<double*>(out_packed);
  a.in_stride = c.C * c.K_in;
  a.out_stride = c.out_len;
  a.C = c.C;
  a.ncols = c.C * nrhs;
  a.R_out = c.R_out;
  a.Rpad = c.Rpad;
  a.K_in = c.K_in;
  a.r_out = c.r_out;
  const int trows = vc->NW * vc->RW;
  a.n_row_tiles = (c.R_out + trows - 1) / trows;
  const int64_t col_tiles = (a.ncols + 64 * vc->CPL - 1) / (64 * vc->CPL);
  a.n_tiles = col_tiles * a.n_row_tiles;
  a.in_table = first ? 1 : 0;
  a.out_table = last ? 1 : 0;
  a.nseg = nseg;
  a.alpha = alpha;
  a.seg = dsegs;
  const int nt = 64 * vc->NW;
  const int64_t resident = (int64_t)occupancy_fn(vc->fn, nt, &vc->occ) * num_cus();
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(a.n_tiles, resident));
  TimedLaunch tl;
  const bool timed = timing_on();
  if (timed) {
    HIP_TRY(hipEventCreate(&tl.a));
    HIP_TRY(hipEventCreate(&tl.b));
    HIP_TRY(hipEventRecord(tl.a, st));
  }
  void* args[] = {&a};
  HIP_TRY(hipLaunchKernel(vc->fn, dim3(grid), dim3(nt), args, 0, st));
  if (timed) {
    HIP_TRY(hipEventRecord(tl.b, st));
    record_timing(tl, A, k, dt, a.ncols, segs, nseg, vc->id);
  }
  return QTT_OK;
}

static void record_timing(TimedLaunch& tl, const qtt_matrix_s* A, int k, int dt, int64_t ncols,
                          const Segment* segs, int nseg, int shape) {
  const CoreDev& c = A->core[k];
  tl.shape = shape;
  const bool first = (k == 0), last = (k == A->d - 1);
  tl.dt = dt;
  tl.pos = (A->d == 1) ? 3 : (first ? 1 : (last ? 2 : 0));
  const double colsd = (double)ncols;
  tl.flops = 2.0 * c.R_out * c.K_in * colsd;
  const double ib = first ? 8.0 : kElemBytes[dt];
  const double ob = last ? 8.0 : kElemBytes[dt];
  tl.bytes = colsd * (c.K_in * ib + (double)c.R_out * ob);
  if (last) {
    bool z = false;
    for (int s = 0; s < nseg; ++s) z = z || segs[s].z != nullptr;
    if (z) tl.bytes += colsd * c.R_out * 8.0;
  }
  g_timed.push_back(tl);
}

// segs: the host copy of the launch's segments (alignment checks, timing);
// dsegs: the same table in device memory, which the kernels read.
static qtt_status_t launch_step(const qtt_matrix_s* A, int k, int dt, int64_t nrhs,
                                const Segment* segs, int nseg, const Segment* dsegs, const void* in_packed,
                                void* out_packed, double alpha, hipStream_t st) {
  const CoreDev& c = A->core[k];
  const bool first = (k == 0), last = (k == A->d - 1);
  const bool in_f64 = first || dt == 0;
  const int in_bytes = in_f64 ? 8 : kElemBytes[dt];
  const int ve = 16 / in_bytes;

  // 16-byte loads need every column start aligned
  bool vec = (c.K_in % ve) == 0;
  if (first) {
    for (int s = 0; s < nseg && vec; ++s)
      vec = (reinterpret_cast<uintptr_t>(segs[s].x) % 16 == 0) && (segs[s].ldx % ve == 0);
  } else {
    vec = vec && (reinterpret_cast<uintptr_t>(in_packed) % 16 == 0);
  }
  int shape = c.tuned[dt];
  if (shape < 0) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(dt, c.R_out, c.K_in, c.r_out, c.C));
    shape = (it != g_tuned.end()) ? it->second : heuristic_shape(c.R_out, c.K_in, dt);
  }
  if (dt == 0 && is_valu_shape(shape))
    return launch_valu(A, k, 0, nrhs, segs, nseg, dsegs, in_packed, out_packed, alpha, shape, st);
  // the resident BF16 kernel serves interior cores that fit it
  const bool resident_ok = dt == 2 && !first && !last && c.R_out <= 256 && c.K_in <= 256 &&
                           c.K_in % 8 == 0 && c.C % 64 == 0 && vec &&
                           reinterpret_cast<uintptr_t>(out_packed) % 16 == 0;
  const bool dma_ok = resident_ok && c.Ksteps[2] <= 8 && c.R_out % 32 == 0;
  if (shape == kBf16Dma32 && !(dma_ok && c.R_out % 64 == 0)) shape = kBf16Dma;
  if (shape == kBf16Dma && !dma_ok) shape = kBf16Resident;
  // the 4x4x4 kernels address the fragment array with 32-bit buffer offsets
  const int64_t m_bytes =
      (int64_t)padded_row_blocks(c.nRB) * c.Ksteps[dt] * 64 * kFragE[dt] * kElemBytes[dt];
  if (shape == kBf16Resident && !resident_ok) shape = heuristic_shape(c.R_out, c.K_in, 1);
  const bool split_ok = dt == 1 && !first && !last && c.fsplit != nullptr && c.fsplit_ks <= 8 &&
                        c.R_out % 64 == 0 && c.R_out <= 256 && c.r_out % 4 == 0 && c.K_in % 8 == 0 &&
                        c.C % 32 == 0 && reinterpret_cast<uintptr_t>(in_packed) % 16 == 0 &&
                        reinterpret_cast<uintptr_t>(out_packed) % 16 == 0;
  if (shape == kF32Split && !split_ok) shape = heuristic_shape(c.R_out, c.K_in, dt);
  // (after the fallbacks above, which can name it)
  if (shape == kValu32) {
    if (dt == 1 && last && !first && c.valu32 != nullptr && c.K_in % 32 == 0 && c.C % 128 == 0 &&
        reinterpret_cast<uintptr_t>(in_packed) % 16 == 0)
      return launch_valu(A, k, 1, nrhs, segs, nseg, dsegs, in_packed, out_packed, alpha, shape, st);
    shape = 2;
  }
  const bool last_ok = dt == 2 && last && !first && c.R_out <= 16 && c.K_in % 8 == 0 && c.Ksteps[2] <= 8 &&
                       c.C % 16 == 0 && vec && reinterpret_cast<uintptr_t>(in_packed) % 16 == 0;
  if (shape == kBf16Last && !last_ok) shape = 2;
  const int tq = smallk_cfg(dt)->TC;
  const bool smallk_ok = first && !last && vec && c.K_in <= 16 && c.K_in % 2 == 0 && c.R_out <= 256 &&
                         c.r_out % 4 == 0 && c.C % tq == 0 && (c.r_out * tq * kElemBytes[dt]) % 16 == 0 &&
                         reinterpret_cast<uintptr_t>(out_packed) % 16 == 0;
  if (shape == kSmallK && !smallk_ok) shape = (dt == 0) ? 67 : 26;   // first-core matrix-core kernels
  const bool smallk_rows = shape == kSmallK && (dt == 2 || dt == 1) && c.K_in <= 8 && c.r_out <= 32 &&
                           c.R_out / c.r_out <= 8 && c.C % 64 == 0;
  KernelCfg* kc = smallk_rows ? smallk_rows_cfg(dt)
                  : (shape == kF32Split) ? f32_split_cfg(c.R_out / 64)
                  : (shape == kSmallK) ? smallk_cfg(dt)
                  : (shape == kBf16Last) ? bf16_last_cfg()
                  : (shape == kBf16Dma) ? bf16_dma_cfg()
                  : (shape == kBf16Dma32) ? bf16_dma32_cfg()
                  : (shape == kBf16Resident) ? bf16_resident_cfg()
                  : vec ? find_cfg(dt, in_f64, true, shape) : find_cfg(dt, in_f64, false, kGenericShape);
  // the streamed 4x4x4 kernels take whole chunks only and address the
  // fragment array with 32-bit buffer offsets
  if (kc && kc->kind == 3 && (c.Ksteps[dt] % (kc->KC / 4) != 0 || m_bytes > INT32_MAX))
    kc = find_cfg(dt, in_f64, true, 21);
  if (!kc) return fail(QTT_ERR_DEVICE, "no kernel for dtype %d shape %d", dt, shape);

  StepArgs a;
  memset(&a, 0, sizeof(a));
  a.M = c.frag[dt];
  a.in = in_packed;
  a.out = out_packed;
  a.C = c.C;
  a.in_stride = c.C * c.K_in;
  a.out_stride = c.out_len;
  a.ncols = c.C * nrhs;
  a.R_out = c.R_out;
  a.K_in = c.K_in;
  a.r_out = c.r_out;
  a.Ksteps = c.Ksteps[dt];
  a.nRB = c.nRB;
  a.n_row_tiles = (c.R_out + kc->TR - 1) / kc->TR;
  const int64_t col_tiles = (a.ncols + kc->TC - 1) / kc->TC;
  a.n_tiles = col_tiles * a.n_row_tiles;
  a.in_table = first ? 1 : 0;
  a.out_table = last ? 1 : 0;
  a.nseg = nseg;
  a.M_bytes = (int32_t)std::min<int64_t>(m_bytes, INT32_MAX);
  a.alpha = alpha;
  a.seg = dsegs;
  if (shape == kF32Split) {       // hi and lo fragment arrays, BF16 steps
    a.M = c.fsplit;
    a.Ksteps = c.fsplit_ks;
    a.M_bytes = c.fsplit_half;
  }

  const int64_t resident = (int64_t)occupancy(kc) * num_cus();
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(a.n_tiles, resident));

  TimedLaunch tl;
  const bool timed = timing_on();
  if (timed) {
    HIP_TRY(hipEventCreate(&tl.a));
    HIP_TRY(hipEventCreate(&tl.b));
    HIP_TRY(hipEventRecord(tl.a, st));
  }
  void* args[] = {&a};
  HIP_TRY(hipLaunchKernel(kc->fn, dim3(grid), dim3(kc->NT), args, 0, st));
  if (timed) {
    HIP_TRY(hipEventRecord(tl.b, st));
    record_timing(tl, A, k, dt, a.ncols, segs, nseg, kc->id);
  }
  return QTT_OK;
}

// ---------------------------------------------------------------------------
// one sweep over a wave of vectors described by segments
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Every apply workspace starts with two segment tables of kMaxSeg entries:
// the sweep's and the diagonal passes' (the two are live at the same time).
static constexpr size_t kSegTableBytes = 2 * kMaxSeg * sizeof(Segment);
static Segment* sweep_table(void* ws) { return static_cast<Segment*>(ws); }
static Segment* diag_table(void* ws) { return static_cast<Segment*>(ws) + kMaxSeg; }
static void* sweep_buffers(void* ws) { return static_cast<char*>(ws) + kSegTableBytes; }

// Write nseg host segments into a device table (captured with the sweep).
static qtt_status_t write_segments(const Segment* segs, int nseg, Segment* table, hipStream_t st) {
  for (int s0 = 0; s0 < nseg; s0 += kSegChunk) {
    SegWriteArgs wa;
    memset(&wa, 0, sizeof(wa));
    wa.dst = table + s0;
    wa.n = std::min(kSegChunk, nseg - s0);
    for (int t = 0; t < wa.n; ++t) wa.seg[t] = segs[s0 + t];
    void* args[] = {&wa};
    HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&seg_write_kernel), dim3(1), dim3(64), args, 0, st));
  }
  return QTT_OK;
}

static size_t wave_buffer_bytes(const qtt_matrix_s* A, int dt, int64_t nrhs) {
  return align256((size_t)A->max_inter * kElemBytes[dt] * (size_t)nrhs);
}

// the two dense FP64 blocks around the sweep of an operator with diagonals
static size_t diag_scratch_bytes(const qtt_matrix_s* A, int64_t nrhs) {
  if (!A->has_diag) return 0;
  return align256((size_t)A->cols * 8 * nrhs) + align256((size_t)A->rows * 8 * nrhs);
}

// workspace of one wave of nrhs vectors: the sweep's two buffers, then the
// diagonal scratch
static size_t wave_total_bytes(const qtt_matrix_s* A, int dt, int64_t nrhs) {
  return kSegTableBytes + (A->d > 1 ? 2 * wave_buffer_bytes(A, dt, nrhs) : 0) + diag_scratch_bytes(A, nrhs);
}

static int64_t wave_capacity(const qtt_matrix_s* A, int dt, size_t ws_bytes) {
  const size_t per = (A->d > 1 ? 2 * (size_t)A->max_inter * kElemBytes[dt] : 0)
                     + (A->has_diag ? (size_t)(A->rows + A->cols) * 8 : 0);
  if (ws_bytes < kSegTableBytes) return 0;
  if (per == 0) return INT64_MAX;
  int64_t w = (int64_t)((ws_bytes - kSegTableBytes) / per);
  while (w > 0 && wave_total_bytes(A, dt, w) > ws_bytes) --w;
  return w;
}

// Fused FP64 pair (core k, core k + 1), see core_pair_f64_kernel.
// configuration ids reported by the launch timing: 90 + 4 (first core) +
// 2 (r_k != 24: the padded rank-32 kernel) + (R_out(k + 1) > 192), one per
// kernel instantiation
static const int kPairShape = 90;
static const int kPairShape32 = 100;   // the same for the FP32 pair kernels
static int64_t frag_bytes(const CoreDev& c, int dt) {
  return (int64_t)padded_row_blocks(c.nRB) * c.Ksteps[dt] * 64 * kFragE[dt] * kElemBytes[dt];
}
static bool pair_ok(const qtt_matrix_s* A, int dt, int k, const Segment* segs, int nseg) {
  if (!((dt == 0 && A->fp64_pair) || (dt == 1 && A->fp32_pair)) || k + 1 > A->d - 2) return false;
  const CoreDev& x = A->core[k];
  const CoreDev& y = A->core[k + 1];
  const bool first = (k == 0);
  const int ra = x.r_out;
  if (!(ra >= 17 && ra <= 32 && x.m == 8 && y.n == 8 && y.K_in == 8 * ra && y.R_out <= 256)) return false;
  if (x.Ksteps[dt] % (first ? 2 : 8) != 0 || y.Ksteps[dt] != (2 * ra + 7) / 8 * 8) return false;
  // 16-byte input loads: 2 FP64 or 4 FP32 values
  if (x.C % 32 != 0 || x.C != y.C || x.K_in % ((first || dt == 0) ? 2 : 4) != 0) return false;
  if (frag_bytes(x, dt) > INT32_MAX || frag_bytes(y, dt) > INT32_MAX) return false;
  if (first)
    for (int s = 0; s < nseg; ++s)
      if (reinterpret_cast<uintptr_t>(segs[s].x) % 16 != 0 || segs[s].ldx % 2 != 0) return false;
  return true;
}
static qtt_status_t launch_pair(const qtt_matrix_s* A, int dt, int k, int64_t nrhs, const Segment* segs,
                                int nseg, const Segment* dsegs, const void* in, void* out, hipStream_t st) {
  const CoreDev& x = A->core[k];
  const CoreDev& y = A->core[k + 1];
  const bool first = (k == 0);
  PairArgs a;
  memset(&a, 0, sizeof(a));
  a.MA = x.frag[dt];
  a.MB = y.frag[dt];
  a.in = static_cast<const double*>(in);
  a.out = static_cast<double*>(out);
  a.in_stride = x.C * x.K_in;
  a.out_stride = y.out_len;
  a.C = x.C;
  a.ncols = x.C * nrhs;
  a.n_tiles = a.ncols / 32;
  a.KsA = x.Ksteps[dt];
  a.KsB = y.Ksteps[dt];
  a.K_inA = x.K_in;
  a.R_outB = y.R_out;
  a.r_outB = y.r_out;
  a.MA_bytes = (int32_t)frag_bytes(x, dt);
  a.MB_bytes = (int32_t)frag_bytes(y, dt);
  a.nseg = first ? nseg : 0;
  a.ra = x.r_out;
  a.seg = dsegs;
  // instantiation: rank of the fused boundary, rows of step k + 1, first core
  // index: 12 dt + 6 first + 2 (0: rank 24, 1: rank 32, 2: padded 17..32) + (rows of core k + 1 > 192)
  static int occ[24] = {};
  static const void* fns[24] = {};
  static std::once_flag fns_once;
  std::call_once(fns_once, [] {
    for (int i = 0; i < 12; ++i) {
      fns[i] = pair_f64_kernel(i);
      fns[12 + i] = pair_f32_kernel(i);
    }
  });
  const int rk = (x.r_out == 24) ? 0 : (x.r_out == 32 ? 1 : 2);
  const int f = (dt == 1 ? 12 : 0) + (first ? 6 : 0) + 2 * rk + (y.R_out > 192 ? 1 : 0);
  // timing id: exact rank 24, else the 256-row kernels (exact or padded)
  const int v = (first ? 4 : 0) + (x.r_out != 24 ? 2 : 0) + (y.R_out > 192 ? 1 : 0);
  const int64_t resident = (int64_t)occupancy_fn(fns[f], 256, &occ[f]) * num_cus();
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(a.n_tiles, resident));
  TimedLaunch tl;
  const bool timed = timing_on();
  if (timed) {
    HIP_TRY(hipEventCreate(&tl.a));
    HIP_TRY(hipEventCreate(&tl.b));
    HIP_TRY(hipEventRecord(tl.a, st));
  }
  void* args[] = {&a};
  HIP_TRY(hipLaunchKernel(fns[f], dim3(grid), dim3(256), args, 0, st));
  if (timed) {
    HIP_TRY(hipEventRecord(tl.b, st));
    tl.dt = dt;
    tl.pos = first ? 1 : 0;
    tl.shape = (dt == 1 ? kPairShape32 : kPairShape) + v;
    tl.flops = 2.0 * ((double)x.R_out * x.K_in + (double)y.R_out * y.K_in) * (double)a.ncols;
    tl.bytes = (double)a.ncols * ((double)x.K_in * (first ? 8 : kElemBytes[dt]) + (double)y.R_out * kElemBytes[dt]);
    g_timed.push_back(tl);
  }
  return QTT_OK;
}

static qtt_status_t sweep(const qtt_matrix_s* A, int dt, int64_t nrhs, const Segment* segs, int nseg,
                          void* ws, double alpha, hipStream_t st) {
  Segment* dsegs = sweep_table(ws);
  qtt_status_t s0 = write_segments(segs, nseg, dsegs, st);
  if (s0 != QTT_OK) return s0;
  void* buf[2] = {sweep_buffers(ws), nullptr};
  if (A->d > 1) buf[1] = static_cast<char*>(buf[0]) + wave_buffer_bytes(A, dt, nrhs);
  int cur = 0;  // buffer holding the latest intermediate (core 0 writes buf[0])
  for (int k = 0; k < A->d;) {
    const void* in = (k == 0) ? nullptr : buf[cur];
    if (pair_ok(A, dt, k, segs, nseg)) {
      qtt_status_t s = launch_pair(A, dt, k, nrhs, segs, nseg, dsegs, in, buf[cur ^ 1], st);
      if (s != QTT_OK) return s;
      cur ^= 1;
      k += 2;
      continue;
    }
    void* out = (k == A->d - 1) ? nullptr : (k == 0 ? buf[0] : buf[cur ^ 1]);
    qtt_status_t s = launch_step(A, k, dt, nrhs, segs, nseg, dsegs, in, out, alpha, st);
    if (s != QTT_OK) return s;
    if (k > 0) cur ^= 1;
    ++k;
  }
  return QTT_OK;
}

static bool graphs_enabled() {
  static int on = [] {
    const char* e = getenv("QTT_GRAPH");
    return (e && e[0] == '0') ? 0 : 1;
  }();
  return on == 1;
}

// One sweep, captured into a graph on first use and replayed afterwards.
// Capture runs on the handle's own stream (the caller's stream may be the
// null stream, which cannot be captured); the graph is launched on the
// caller's stream.  Timed runs launch directly (per-launch events).
static qtt_status_t sweep_graph(const qtt_matrix_s* A, int dt, int64_t nrhs, const Segment* segs, int nseg,
                                void* ws, double alpha, hipStream_t st) {
  if (!graphs_enabled() || timing_on()) return sweep(A, dt, nrhs, segs, nseg, ws, alpha, st);
  std::string key;
  auto put = [&](const void* p, size_t n) { key.append(static_cast<const char*>(p), n); };
  put(&dt, sizeof dt);
  put(&nrhs, sizeof nrhs);
  put(&alpha, sizeof alpha);
  put(&ws, sizeof ws);
  put(&A->tune_gen, sizeof A->tune_gen);
  const int64_t gen = g_tune_gen.load();
  put(&gen, sizeof gen);
  for (int i = 0; i < nseg; ++i) put(&segs[i], sizeof(Segment));
  std::lock_guard<std::mutex> lk(A->graph_mu);
  for (size_t i = 0; i < A->graphs.size(); ++i) {
    if (A->graphs[i].key == key) {
      qtt_matrix_s::Graph g = A->graphs[i];
      A->graphs.erase(A->graphs.begin() + i);
      A->graphs.push_back(g);
      HIP_TRY(hipGraphLaunch(g.exec, st));
      HIP_TRY(hipEventRecord(g.done, st));
      return QTT_OK;
    }
  }
  // first use: run directly (this also settles every lazily queried launch
  // parameter), then capture the same launches for later calls
  qtt_status_t s0 = sweep(A, dt, nrhs, segs, nseg, ws, alpha, st);
  if (s0 != QTT_OK) return s0;
  if (A->cap_stream == nullptr) HIP_TRY(hipStreamCreateWithFlags(&A->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(A->cap_stream, hipStreamCaptureModeThreadLocal));
  qtt_status_t s = sweep(A, dt, nrhs, segs, nseg, ws, alpha, A->cap_stream);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(A->cap_stream, &graph);
  if (s != QTT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(QTT_ERR_DEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(QTT_ERR_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
  }
  hipEvent_t done = nullptr;
  e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return fail(QTT_ERR_DEVICE, "hipEventCreate failed: %s", hipGetErrorString(e));
  }
  if (A->graphs.size() >= kMaxGraphs) {
    destroy_graph(A->graphs.front());
    A->graphs.erase(A->graphs.begin());
  }
  A->graphs.push_back({key, graph, exec, done});
  return QTT_OK;
}

// y = z + alpha (a x + b . K (wc . x)) for a wave: scale the inputs into the
// first scratch block, sweep K from it into the second, then the epilogue.
// The scratch sits after the sweep buffers of a full wave (cap vectors), so
// it never overlaps the buffers of this wave.
static qtt_status_t diag_sweep(const qtt_matrix_s* A, int dt, int64_t nrhs, int64_t cap,
                               const std::vector<Segment>& segs, void* ws, double alpha, hipStream_t st,
                               bool use_graph) {
  char* base = static_cast<char*>(sweep_buffers(ws)) + (A->d > 1 ? 2 * wave_buffer_bytes(A, dt, cap) : 0);
  double* S1 = reinterpret_cast<double*>(base);
  double* S2 = reinterpret_cast<double*>(base + align256((size_t)A->cols * 8 * cap));
  DiagArgs da;
  memset(&da, 0, sizeof(da));
  Segment* dtab = diag_table(ws);
  qtt_status_t sw = write_segments(segs.data(), (int)segs.size(), dtab, st);
  if (sw != QTT_OK) return sw;
  da.seg = dtab;
  da.nseg = (int32_t)segs.size();
  da.ncol = nrhs;
  auto grid = [&](int64_t rows) {
    return dim3((unsigned)std::min<int64_t>(256, std::max<int64_t>(1, (rows + 255) / 256)),
                (unsigned)std::min<int64_t>(nrhs, 65535));
  };
  da.rows = A->cols;
  da.d = A->diag_wc;
  da.S = S1;
  void* args[] = {&da};
  HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&diag_in_kernel), grid(A->cols), dim3(256), args, 0, st));
  Segment one;
  one.x = S1;
  one.y = S2;
  one.z = nullptr;
  one.ldx = A->cols;
  one.ldy = A->rows;
  one.ldz = 0;
  one.rhs_begin = 0;
  qtt_status_t s = use_graph ? sweep_graph(A, dt, nrhs, &one, 1, ws, 1.0, st)
                             : sweep(A, dt, nrhs, &one, 1, ws, 1.0, st);
  if (s != QTT_OK) return s;
  da.rows = A->rows;
  da.d = A->diag_b;
  da.S = S2;
  da.a = A->diag_a;
  da.alpha = alpha;
  HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&diag_out_kernel), grid(A->rows), dim3(256), args, 0, st));
  return QTT_OK;
}

// A block of vectors before splitting into waves.
struct Block {
  const double* x;
  double* y;
  const double* z;
  int64_t ldx, ldy, ldz, width;
};

// Run y = z + alpha * A x over blocks, in waves bounded by the workspace and
// by the segment-table size.  use_graph = false launches every sweep directly
// (no graph capture or instantiation, which allocate).
static qtt_status_t run_blocks(const qtt_matrix_s* A, int dt, const std::vector<Block>& blocks,
                               void* ws, size_t ws_bytes, double alpha, hipStream_t st,
                               bool use_graph = true) {
  int64_t total = 0;
  for (auto& b : blocks) total += b.width;
  if (total == 0) return QTT_OK;
  const int64_t cap = wave_capacity(A, dt, ws_bytes);
  if (cap < 1) {
    size_t need = wave_total_bytes(A, dt, 1);
    return fail(QTT_ERR_WORKSPACE, "workspace of %zu bytes is below the one-vector minimum %zu", ws_bytes, need);
  }
  std::vector<Segment> segs;
  int64_t in_wave = 0;
  auto flush = [&]() -> qtt_status_t {
    if (in_wave == 0) return QTT_OK;
    qtt_status_t s = A->has_diag ? diag_sweep(A, dt, in_wave, cap, segs, ws, alpha, st, use_graph)
                     : use_graph ? sweep_graph(A, dt, in_wave, segs.data(), (int)segs.size(), ws, alpha, st)
                                 : sweep(A, dt, in_wave, segs.data(), (int)segs.size(), ws, alpha, st);
    segs.clear();
    in_wave = 0;
    return s;
  };
  for (auto& b : blocks) {
    int64_t done = 0;
    while (done < b.width) {
      if (in_wave == cap || (int)segs.size() == kMaxSeg) {
        qtt_status_t s = flush();
        if (s != QTT_OK) return s;
      }
      const int64_t take = std::min(b.width - done, cap - in_wave);
      Segment sg;
      sg.x = b.x + done * b.ldx;
      sg.y = b.y + done * b.ldy;
      sg.z = b.z ? b.z + done * b.ldz : nullptr;
      sg.ldx = b.ldx;
      sg.ldy = b.ldy;
      sg.ldz = b.ldz;
      sg.rhs_begin = in_wave;
      segs.push_back(sg);
      in_wave += take;
      done += take;
    }
  }
  return flush();
}

static bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bn && pb < pa + an;
}

static qtt_status_t check_dtype(const qtt_matrix_s* A, qtt_dtype_t t, int* dt) {
  *dt = dt_index(t);
  if (*dt < 0) return fail(QTT_ERR_INVALID_ARG, "unknown compute dtype %d", (int)t);
  if (!(A->dtypes & (uint32_t)t)) return fail(QTT_ERR_DTYPE, "matrix was not loaded with dtype %d", (int)t);
  return QTT_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* qtt_status_string(qtt_status_t s) {
  switch (s) {
    case QTT_OK: return "ok";
    case QTT_ERR_INVALID_ARG: return "invalid argument";
    case QTT_ERR_SHAPE: return "inconsistent shape";
    case QTT_ERR_OUT_OF_MEMORY: return "out of device memory";
    case QTT_ERR_DEVICE: return "HIP error";
    case QTT_ERR_NOT_CONVERGED: return "not converged";
    case QTT_ERR_NONFINITE: return "non-finite residual";
    case QTT_ERR_WORKSPACE: return "workspace too small";
    case QTT_ERR_DTYPE: return "dtype not loaded";
    case QTT_ERR_RANK: return "rank cap reached";
  }
  return "unknown status";
}

const char* qtt_last_error(void) { return g_last_error.c_str(); }

qtt_status_t qtt_matrix_load(int32_t d, const int64_t* ranks, const int64_t* m, const int64_t* n,
                             const double* const* cores, uint32_t dtypes, qtt_matrix_t* out) {
  if (out == nullptr) return fail(QTT_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (d < 1 || d > 64) return fail(QTT_ERR_INVALID_ARG, "d = %d outside [1, 64]", d);
  if (!ranks || !m || !n || !cores) return fail(QTT_ERR_INVALID_ARG, "null shape or core array");
  if (dtypes == 0 || (dtypes & ~7u)) return fail(QTT_ERR_INVALID_ARG, "dtypes must be a non-empty OR of QTT_FP64/FP32/BF16");
  if (ranks[0] != 1 || ranks[d] != 1) return fail(QTT_ERR_SHAPE, "boundary ranks must be 1");
  for (int k = 0; k < d; ++k) {
    if (ranks[k + 1] < 1 || m[k] < 1 || n[k] < 1) return fail(QTT_ERR_SHAPE, "core %d: ranks and modes must be >= 1", k);
    if (!cores[k]) return fail(QTT_ERR_INVALID_ARG, "core %d pointer is null", k);
    if (ranks[k] * m[k] > (1 << 20) || ranks[k] * n[k] > (1 << 20) || ranks[k + 1] * m[k] > (1 << 20))
      return fail(QTT_ERR_SHAPE, "core %d too large", k);
  }
  // vector lengths (guard overflow)
  double rows = 1, cols = 1;
  for (int k = 0; k < d; ++k) { rows *= (double)m[k]; cols *= (double)n[k]; }
  if (rows > 4e15 || cols > 4e15) return fail(QTT_ERR_SHAPE, "vector length overflows");

  qtt_matrix_s* A = new qtt_matrix_s();
  A->d = d;
  A->ranks.assign(ranks, ranks + d + 1);
  A->m.assign(m, m + d);
  A->n.assign(n, n + d);
  A->rows = 1;
  A->cols = 1;
  for (int k = 0; k < d; ++k) { A->rows *= m[k]; A->cols *= n[k]; }
  A->max_rank = *std::max_element(ranks, ranks + d + 1);
  A->dtypes = dtypes;
  (void)hipGetDevice(&A->device);
  A->core.resize(d);

  for (int k = 0; k < d; ++k) {
    CoreDev& c = A->core[k];
    c.r_in = (int)ranks[k];
    c.r_out = (int)ranks[k + 1];
    c.m = (int)m[k];
    c.n = (int)n[k];
    c.R_out = c.r_out * c.m;
    c.K_in = c.r_in * c.n;
    int64_t lo = 1, hi = 1;
    for (int l = 0; l < k; ++l) lo *= m[l];
    for (int l = k + 1; l < d; ++l) hi *= n[l];
    c.C = lo * hi;
    c.out_len = (int64_t)c.r_out * c.C * c.m;
    c.nRB = (c.R_out + 15) / 16;
    for (int t = 0; t < 3; ++t) { c.frag[t] = nullptr; c.Ksteps[t] = 0; c.tuned[t] = -1; }
    c.valu = nullptr;
    c.valu1 = nullptr;
    c.g64 = nullptr;
    c.Rpad = 0;
    if (k < d - 1) A->max_inter = std::max(A->max_inter, c.out_len);
  }

  // re-layout: fragment (row block rb, step s, lane l, element e) holds
  // M_k(16 rb + l mod 16, KSTEP s + E (l div 16) + e), zero outside the matrix.
  for (int k = 0; k < d; ++k) {
    CoreDev& c = A->core[k];
    const double* G = cores[k];
    for (int t = 0; t < 3; ++t) {
      if (!(dtypes & (1u << t))) continue;
      const int KS = kKstep[t], E = kFragE[t];
      int Ksteps = (c.K_in + KS - 1) / KS;
      // FP64 and FP32 cores of more than 8 steps get zero steps up to a multiple of 8,
      // the chunk of the streamed 4x4x4 kernels (so any rank can use them;
      // every kernel reads input indices past K_in as zeros or as finite data
      // multiplied by these zero core values)
      if (t <= 1 && Ksteps > 8) Ksteps = (Ksteps + 7) / 8 * 8;
      c.Ksteps[t] = Ksteps;
      // row blocks padded with zeros so that every tile height of the
      // registry covers a whole number of tiles: kernels may then read the
      // row blocks of any tile without bounds tests
      const int nRBpad = padded_row_blocks(c.nRB);
      const size_t nel = (size_t)nRBpad * Ksteps * 64 * E;
      std::vector<double> h(nel, 0.0);
      for (int rb = 0; rb < c.nRB; ++rb)
        for (int s = 0; s < Ksteps; ++s)
          for (int l = 0; l < 64; ++l)
            for (int e = 0; e < E; ++e) {
              const int row = 16 * rb + (l & 15);
              const int kap = KS * s + E * (l >> 4) + e;
              if (row >= c.R_out || kap >= c.K_in) continue;
              const int ak = row % c.r_out, ik = row / c.r_out;   // row = a_k + r_k i_k
              const int ap = kap % c.r_in, jk = kap / c.r_in;     // kap = a_{k-1} + r_{k-1} j_k
              h[(((size_t)rb * Ksteps + s) * 64 + l) * E + e] =
                  G[(((size_t)ap * c.m + ik) * c.n + jk) * c.r_out + ak];
            }
      const size_t bytes = nel * kElemBytes[t];
      void* dptr = nullptr;
      if (hipMalloc(&dptr, std::max<size_t>(bytes, 256)) != hipSuccess) {
        qtt_matrix_free(A);
        return fail(QTT_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes for core %d failed", bytes, k);
      }
      c.frag[t] = dptr;
      hipError_t e;
      if (t == 0) {
        e = hipMemcpy(dptr, h.data(), bytes, hipMemcpyHostToDevice);
      } else if (t == 1) {
        std::vector<float> f(nel);
        for (size_t i = 0; i < nel; ++i) f[i] = (float)h[i];
        e = hipMemcpy(dptr, f.data(), bytes, hipMemcpyHostToDevice);
      } else {
        std::vector<uint16_t> b(nel);
        for (size_t i = 0; i < nel; ++i) b[i] = f64_to_bf16_rne(h[i]);
        e = hipMemcpy(dptr, b.data(), bytes, hipMemcpyHostToDevice);
      }
      if (e != hipSuccess) {
        qtt_matrix_free(A);
        return fail(QTT_ERR_DEVICE, "hipMemcpy of core %d failed: %s", k, hipGetErrorString(e));
      }
    }
  }
  // FP32 cores split for configuration kF32Split: v = (float) M_k(row, kap),
  // hi = bf16(v), lo = bf16(v - hi), each array in the BF16 fragment layout
  if (dtypes & QTT_FP32) {
    for (int k = 0; k < d; ++k) {
      CoreDev& c = A->core[k];
      if (c.K_in > 256 || c.K_in % 8 != 0) continue;
      const double* G = cores[k];
      const int KS = kKstep[2], E = kFragE[2];
      const int Ksteps = (c.K_in + KS - 1) / KS;
      const size_t nel = (size_t)padded_row_blocks(c.nRB) * Ksteps * 64 * E;
      std::vector<uint16_t> b(2 * nel, 0);
      for (int rb = 0; rb < c.nRB; ++rb)
        for (int s = 0; s < Ksteps; ++s)
          for (int l = 0; l < 64; ++l)
            for (int e = 0; e < E; ++e) {
              const int row = 16 * rb + (l & 15);
              const int kap = KS * s + E * (l >> 4) + e;
              if (row >= c.R_out || kap >= c.K_in) continue;
              const int ak = row % c.r_out, ik = row / c.r_out;
              const int ap = kap % c.r_in, jk = kap / c.r_in;
              const float v = (float)G[(((size_t)ap * c.m + ik) * c.n + jk) * c.r_out + ak];
              const uint16_t hi = f32_to_bf16_rne(v);
              const float hv = __builtin_bit_cast(float, (uint32_t)hi << 16);
              const size_t at = (((size_t)rb * Ksteps + s) * 64 + l) * E + e;
              b[at] = hi;
              b[nel + at] = f32_to_bf16_rne(v - hv);
            }
      void* dptr = nullptr;
      if (hipMalloc(&dptr, std::max<size_t>(2 * nel * 2, 256)) != hipSuccess) {
        qtt_matrix_free(A);
        return fail(QTT_ERR_OUT_OF_MEMORY, "hipMalloc for the split FP32 copy of core %d failed", k);
      }
      c.fsplit = dptr;
      c.fsplit_ks = Ksteps;
      c.fsplit_half = (int32_t)(nel * 2);
      hipError_t er = hipMemcpy(dptr, b.data(), 2 * nel * 2, hipMemcpyHostToDevice);
      if (er != hipSuccess) {
        qtt_matrix_free(A);
        return fail(QTT_ERR_DEVICE, "hipMemcpy of core %d failed: %s", k, hipGetErrorString(er));
      }
    }
  }
  // FP32 vector-ALU copy of the last core (groups of 8), values (float) M_d
  if ((dtypes & QTT_FP32) && d > 1) {
    CoreDev& c = A->core[d - 1];
    const double* G = cores[d - 1];
    if (c.K_in % 32 == 0) {
      const int Rpad = valu_padded_rows(c.R_out);
      const size_t nel = (size_t)c.K_in * Rpad;
      std::vector<float> h(nel, 0.f);
      for (int row = 0; row < c.R_out; ++row)
        for (int kap = 0; kap < c.K_in; ++kap) {
          const int ak = row % c.r_out, ik = row / c.r_out;
          const int ap = kap % c.r_in, jk = kap / c.r_in;
          h[((size_t)(kap / 8) * Rpad + row) * 8 + kap % 8] =
              (float)G[(((size_t)ap * c.m + ik) * c.n + jk) * c.r_out + ak];
        }
      void* dptr = nullptr;
      if (hipMalloc(&dptr, std::max<size_t>(nel * 4, 256)) != hipSuccess) {
        qtt_matrix_free(A);
        return fail(QTT_ERR_OUT_OF_MEMORY, "hipMalloc for the FP32 vector-ALU copy of core %d failed", d - 1);
      }
      c.valu32 = static_cast<float*>(dptr);
      c.Rpad = Rpad;
      hipError_t er = hipMemcpy(dptr, h.data(), nel * 4, hipMemcpyHostToDevice);
      if (er != hipSuccess) {
        qtt_matrix_free(A);
        return fail(QTT_ERR_DEVICE, "hipMemcpy of core %d failed: %s", d - 1, hipGetErrorString(er));
      }
    }
  }
  // FP64 vector-ALU copies: Mv[(g * Rpad + row) * G + e] = M_k(row, G g + e)
  if (dtypes & QTT_FP64) {
    for (int k = 0; k < d; ++k) {
      CoreDev& c = A->core[k];
      const double* G = cores[k];
      c.Rpad = valu_padded_rows(c.R_out);
      for (int gs : {8, 1}) {
        if (c.K_in % gs) continue;
        const size_t nel = (size_t)c.K_in * c.Rpad;
        std::vector<double> h(nel, 0.0);
        for (int row = 0; row < c.R_out; ++row)
          for (int kap = 0; kap < c.K_in; ++kap) {
            const int ak = row % c.r_out, ik = row / c.r_out;
            const int ap = kap % c.r_in, jk = kap / c.r_in;
            h[((size_t)(kap / gs) * c.Rpad + row) * gs + kap % gs] =
                G[(((size_t)ap * c.m + ik) * c.n + jk) * c.r_out + ak];
          }
        void* dptr = nullptr;
        if (hipMalloc(&dptr, std::max<size_t>(nel * 8, 256)) != hipSuccess) {
          qtt_matrix_free(A);
          return fail(QTT_ERR_OUT_OF_MEMORY, "hipMalloc for the FP64 vector-ALU copy of core %d failed", k);
        }
        (gs == 8 ? c.valu : c.valu1) = static_cast<double*>(dptr);
        hipError_t er = hipMemcpy(dptr, h.data(), nel * 8, hipMemcpyHostToDevice);
        if (er != hipSuccess) {
          qtt_matrix_free(A);
          return fail(QTT_ERR_DEVICE, "hipMemcpy of core %d failed: %s", k, hipGetErrorString(er));
        }
      }
    }
  }
  // FP64 cores as given (the compressed matrix-vector product reads them)
  if (dtypes & QTT_FP64) {
    for (int k = 0; k < d; ++k) {
      CoreDev& c = A->core[k];
      const size_t nel = (size_t)c.r_in * c.m * c.n * c.r_out;
      void* dptr = nullptr;
      if (hipMalloc(&dptr, std::max<size_t>(nel * 8, 256)) != hipSuccess) {
        qtt_matrix_free(A);
        return fail(QTT_ERR_OUT_OF_MEMORY, "hipMalloc for the FP64 copy of core %d failed", k);
      }
      c.g64 = static_cast<double*>(dptr);
      hipError_t er = hipMemcpy(dptr, cores[k], nel * 8, hipMemcpyHostToDevice);
      if (er != hipSuccess) {
        qtt_matrix_free(A);
        return fail(QTT_ERR_DEVICE, "hipMemcpy of core %d failed: %s", k, hipGetErrorString(er));
      }
    }
  }
  *out = A;
  return QTT_OK;
}

qtt_status_t qtt_matrix_free(qtt_matrix_t A) {
  if (A == nullptr) return QTT_OK;
  drop_graphs(A);
  if (A->cap_stream) (void)hipStreamDestroy(A->cap_stream);
  if (A->diag_b) (void)hipFree(A->diag_b);
  if (A->diag_wc) (void)hipFree(A->diag_wc);
  for (auto& c : A->core) {
    for (int t = 0; t < 3; ++t)
      if (c.frag[t]) (void)hipFree(c.frag[t]);
    if (c.valu) (void)hipFree(c.valu);
    if (c.valu1) (void)hipFree(c.valu1);
    if (c.g64) (void)hipFree(c.g64);
    if (c.fsplit) (void)hipFree(c.fsplit);
    if (c.valu32) (void)hipFree(c.valu32);
  }
  delete A;
  return QTT_OK;
}

qtt_status_t qtt_matrix_set_diagonals(qtt_matrix_t A, double a, const double* b, const double* wc) {
  if (!valid_handle(A)) return fail(QTT_ERR_INVALID_ARG, "null handle");
  if (!std::isfinite(a)) return fail(QTT_ERR_INVALID_ARG, "a is not finite");
  if (a != 0.0 && A->rows != A->cols) return fail(QTT_ERR_SHAPE, "a I needs a square matrix");
  for (int64_t i = 0; b && i < A->rows; ++i)
    if (!std::isfinite(b[i])) return fail(QTT_ERR_INVALID_ARG, "b[%lld] is not finite", (long long)i);
  for (int64_t i = 0; wc && i < A->cols; ++i)
    if (!std::isfinite(wc[i])) return fail(QTT_ERR_INVALID_ARG, "wc[%lld] is not finite", (long long)i);
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  HIP_TRY(hipSetDevice(A->device));
  auto upload = [&](const double* h, int64_t n, double** dptr) -> qtt_status_t {
    if (*dptr) (void)hipFree(*dptr);
    *dptr = nullptr;
    if (!h) return QTT_OK;
    if (hipMalloc(reinterpret_cast<void**>(dptr), std::max<size_t>(n * 8, 256)) != hipSuccess) {
      *dptr = nullptr;
      return fail(QTT_ERR_OUT_OF_MEMORY, "hipMalloc of %lld diagonal entries failed", (long long)n);
    }
    HIP_TRY(hipMemcpy(*dptr, h, n * 8, hipMemcpyHostToDevice));
    return QTT_OK;
  };
  qtt_status_t s = upload(b, A->rows, &A->diag_b);
  if (s == QTT_OK) s = upload(wc, A->cols, &A->diag_wc);
  (void)hipSetDevice(cur);
  if (s != QTT_OK) {
    A->has_diag = false;
    return s;
  }
  A->diag_a = a;
  A->has_diag = (a != 0.0) || b || wc;
  drop_graphs(A);
  return QTT_OK;
}

qtt_status_t qtt_matrix_info(qtt_matrix_t A, int32_t* d, int64_t* rows, int64_t* cols,
                             int64_t* max_rank, uint32_t* dtypes) {
  if (!valid_handle(A)) return fail(QTT_ERR_INVALID_ARG, "null handle");
  if (d) *d = A->d;
  if (rows) *rows = A->rows;
  if (cols) *cols = A->cols;
  if (max_rank) *max_rank = A->max_rank;
  if (dtypes) *dtypes = A->dtypes;
  return QTT_OK;
}

qtt_status_t qtt_matrix_shape(qtt_matrix_t A, int64_t* ranks, int64_t* m, int64_t* n) {
  if (!valid_handle(A)) return fail(QTT_ERR_INVALID_ARG, "null handle");
  for (int k = 0; k <= A->d && ranks; ++k) ranks[k] = A->ranks[k];
  for (int k = 0; k < A->d; ++k) {
    if (m) m[k] = A->m[k];
    if (n) n[k] = A->n[k];
  }
  return QTT_OK;
}

qtt_status_t qtt_workspace_bytes(qtt_matrix_t A, qtt_dtype_t compute, int64_t nrhs, size_t* bytes) {
  if (!valid_handle(A) || !bytes) return fail(QTT_ERR_INVALID_ARG, "null handle or output");
  if (nrhs < 0) return fail(QTT_ERR_INVALID_ARG, "nrhs < 0");
  int dt;
  qtt_status_t s = check_dtype(A, compute, &dt);
  if (s != QTT_OK) return s;
  *bytes = wave_total_bytes(A, dt, std::max<int64_t>(nrhs, 1));
  return QTT_OK;
}

qtt_status_t qtt_apply(qtt_matrix_t A, qtt_dtype_t compute, int64_t nrhs, const double* X, int64_t ldx,
                       double* Y, int64_t ldy, void* ws, size_t ws_bytes, void* stream) {
  if (!valid_handle(A)) return fail(QTT_ERR_INVALID_ARG, "null handle");
  int dt;
  qtt_status_t s = check_dtype(A, compute, &dt);
  if (s != QTT_OK) return s;
  if (nrhs < 0) return fail(QTT_ERR_INVALID_ARG, "nrhs < 0");
  if (nrhs == 0) return QTT_OK;
  if (!X || !Y) return fail(QTT_ERR_INVALID_ARG, "X or Y is null");
  if (ldx < A->cols || ldy < A->rows) return fail(QTT_ERR_INVALID_ARG, "ldx < N or ldy < M");
  if (wave_total_bytes(A, dt, 1) > 0 && !ws) return fail(QTT_ERR_INVALID_ARG, "workspace is null");
  const size_t xb = ((size_t)(nrhs - 1) * ldx + A->cols) * 8, yb = ((size_t)(nrhs - 1) * ldy + A->rows) * 8;
  if (overlaps(X, xb, Y, yb)) return fail(QTT_ERR_INVALID_ARG, "X and Y overlap");
  if (ws && (overlaps(ws, ws_bytes, X, xb) || overlaps(ws, ws_bytes, Y, yb)))
    return fail(QTT_ERR_INVALID_ARG, "workspace overlaps X or Y");
  std::vector<Block> blocks{{X, Y, nullptr, ldx, ldy, 0, nrhs}};
  return run_blocks(A, dt, blocks, ws, ws_bytes, 1.0, static_cast<hipStream_t>(stream));
}

qtt_status_t qtt_apply_batched(qtt_matrix_t A, qtt_dtype_t compute, int32_t nblocks, const int64_t* widths,
                               const double* const* X, const int64_t* ldx, double* const* Y,
                               const int64_t* ldy, void* ws, size_t ws_bytes, void* stream) {
  if (!valid_handle(A)) return fail(QTT_ERR_INVALID_ARG, "null handle");
  int dt;
  qtt_status_t s = check_dtype(A, compute, &dt);
  if (s != QTT_OK) return s;
  if (nblocks < 0) return fail(QTT_ERR_INVALID_ARG, "nblocks < 0");
  if (nblocks == 0) return QTT_OK;
  if (!widths || !X || !ldx || !Y || !ldy) return fail(QTT_ERR_INVALID_ARG, "null block array");
  if (wave_total_bytes(A, dt, 1) > 0 && !ws) return fail(QTT_ERR_INVALID_ARG, "workspace is null");
  std::vector<Block> blocks;
  std::vector<std::pair<const void*, size_t>> xs, ys;
  for (int b = 0; b < nblocks; ++b) {
    if (widths[b] < 0) return fail(QTT_ERR_INVALID_ARG, "block %d has negative width", b);
    if (widths[b] == 0) continue;
    if (!X[b] || !Y[b]) return fail(QTT_ERR_INVALID_ARG, "block %d has a null pointer", b);
    if (ldx[b] < A->cols || ldy[b] < A->rows) return fail(QTT_ERR_INVALID_ARG, "block %d: ld too small", b);
    blocks.push_back({X[b], Y[b], nullptr, ldx[b], ldy[b], 0, widths[b]});
    xs.push_back({X[b], ((size_t)(widths[b] - 1) * ldx[b] + A->cols) * 8});
    ys.push_back({Y[b], ((size_t)(widths[b] - 1) * ldy[b] + A->rows) * 8});
  }
  for (auto& y : ys) {
    for (auto& x : xs)
      if (overlaps(y.first, y.second, x.first, x.second)) return fail(QTT_ERR_INVALID_ARG, "an output block overlaps an input block");
    if (ws && overlaps(ws, ws_bytes, y.first, y.second)) return fail(QTT_ERR_INVALID_ARG, "workspace overlaps an output block");
  }
  return run_blocks(A, dt, blocks, ws, ws_bytes, 1.0, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// Workspace of qtt_apply_noalloc: a file-scope device array, one copy per GPU
// for the life of the process.  Host code never passes the array's name to a
// kernel or copy (on the host it is only a stand-in symbol); it uses the
// device address that hipGetSymbolAddress returns for the current device.
static constexpr size_t kScratchBytes = size_t(512) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

static qtt_status_t scratch_address(int device, void** ptr) {
  if (device < 0 || device >= 64) return fail(QTT_ERR_DEVICE, "device %d out of the supported range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(QTT_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device,
                  hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return QTT_OK;
}

extern "C" {

qtt_status_t qtt_apply_noalloc(qtt_matrix_t A, qtt_dtype_t compute, int64_t nrhs, const double* X, int64_t ldx,
                               double* Y, int64_t ldy, void* stream) {
  if (!valid_handle(A)) return fail(QTT_ERR_INVALID_ARG, "null handle");
  int dt;
  qtt_status_t s = check_dtype(A, compute, &dt);
  if (s != QTT_OK) return s;
  if (nrhs < 0) return fail(QTT_ERR_INVALID_ARG, "nrhs < 0");
  if (nrhs == 0) return QTT_OK;
  if (!X || !Y) return fail(QTT_ERR_INVALID_ARG, "X or Y is null");
  if (ldx < A->cols || ldy < A->rows) return fail(QTT_ERR_INVALID_ARG, "ldx < N or ldy < M");
  const size_t need = wave_total_bytes(A, dt, 1);
  if (need > kScratchBytes)
    return fail(QTT_ERR_WORKSPACE,
                "one vector needs %zu bytes of workspace, above the %zu-byte static workspace of qtt_apply_noalloc",
                need, kScratchBytes);
  const size_t xb = ((size_t)(nrhs - 1) * ldx + A->cols) * 8, yb = ((size_t)(nrhs - 1) * ldy + A->rows) * 8;
  if (overlaps(X, xb, Y, yb)) return fail(QTT_ERR_INVALID_ARG, "X and Y overlap");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != A->device) return fail(QTT_ERR_INVALID_ARG, "the current device %d is not the handle's %d", dev, A->device);
  void* ws = nullptr;
  s = scratch_address(dev, &ws);
  if (s != QTT_OK) return s;
  std::vector<Block> blocks{{X, Y, nullptr, ldx, ldy, 0, nrhs}};
  g_timing_off = true;
  s = run_blocks(A, dt, blocks, ws, kScratchBytes, 1.0, static_cast<hipStream_t>(stream), false);
  g_timing_off = false;
  return s;
}

qtt_status_t qtt_autotune(qtt_matrix_t A, qtt_dtype_t compute, int64_t nrhs, const double* X, int64_t ldx,
                          double* Y, int64_t ldy, void* ws, size_t ws_bytes, void* stream) {
  qtt_status_t s = qtt_apply(A, compute, nrhs, X, ldx, Y, ldy, ws, ws_bytes, stream);  // validates, warms up
  if (s != QTT_OK) return s;
  drop_graphs(A);
  int dt = dt_index(compute);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t cap = wave_capacity(A, dt, ws_bytes);
  const int64_t w = std::min<int64_t>(nrhs, cap);
  Segment sg;
  sg.x = X; sg.y = Y; sg.z = nullptr; sg.ldx = ldx; sg.ldy = ldy; sg.ldz = 0; sg.rhs_begin = 0;
  void* b0 = sweep_buffers(ws);
  void* buf[2] = {b0, (A->d > 1) ? static_cast<char*>(b0) + wave_buffer_bytes(A, dt, w) : nullptr};
  Segment* dsegs = sweep_table(ws);
  s = write_segments(&sg, 1, dsegs, st);
  if (s != QTT_OK) return s;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const bool was_timing = g_timing;
  g_timing = false;
  for (int k = 0; k < A->d; ++k) {
    CoreDev& c = A->core[k];
    const void* in = (k == 0) ? nullptr : buf[(k - 1) & 1];
    void* out = (k == A->d - 1) ? nullptr : buf[k & 1];
    float best = 1e30f;
    int best_id = -1;
    const bool in_f64 = (k == 0) || dt == 0;
    std::vector<int> ids = shape_ids(dt, in_f64);
    if (dt == 2 && k > 0 && k < A->d - 1) {
      ids.push_back(kBf16Resident);
      ids.push_back(kBf16Dma);
      ids.push_back(kBf16Dma32);
    }
    if (k == 0 && A->d > 1) ids.push_back(kSmallK);
    if (dt == 2 && k == A->d - 1 && k > 0) ids.push_back(kBf16Last);
    if (dt == 1 && k == A->d - 1 && k > 0) ids.push_back(kValu32);
    if (dt == 0)
      for (auto& vc : valu_registry())
        if (vc.G == 1 || c.K_in % vc.G == 0) ids.push_back(vc.id);
    for (int id : ids) {
      c.tuned[dt] = id;
      for (int rep = 0; rep < 2; ++rep) {           // warm-up + timed
        HIP_TRY(hipEventRecord(e0, st));
        for (int it = 0; it < 3; ++it) {
          s = launch_step(A, k, dt, w, &sg, 1, dsegs, in, out, 1.0, st);
          if (s != QTT_OK) { g_timing = was_timing; return s; }
        }
        HIP_TRY(hipEventRecord(e1, st));
      }
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (tune_log())
        fprintf(stderr, "qtt_autotune dtype %d core %d (%d x %d, %lld cols) shape %d: %.4f ms\n", dt, k,
                c.R_out, c.K_in, (long long)(c.C * w), id, ms / 3);
      if (ms < best) { best = ms; best_id = id; }
    }
    c.tuned[dt] = best_id;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(dt, c.R_out, c.K_in, c.r_out, c.C)] = best_id;
    ++g_tune_gen;
  }
  if (dt <= 1) {
    // fused pairs against the standard sweep
    bool& pair = (dt == 0) ? A->fp64_pair : A->fp32_pair;
    float ms_mode[2] = {0, 0};
    for (int mode = 0; mode < 2; ++mode) {
      pair = (mode == 1);
      for (int rep = 0; rep < 2; ++rep) {
        HIP_TRY(hipEventRecord(e0, st));
        for (int it = 0; it < 2; ++it) {
          s = sweep(A, dt, w, &sg, 1, ws, 1.0, st);
          if (s != QTT_OK) { g_timing = was_timing; return s; }
        }
        HIP_TRY(hipEventRecord(e1, st));
      }
      HIP_TRY(hipEventSynchronize(e1));
      HIP_TRY(hipEventElapsedTime(&ms_mode[mode], e0, e1));
    }
    pair = ms_mode[1] < ms_mode[0];
    if (tune_log())
      fprintf(stderr, "qtt_autotune dtype %d whole sweep: standard %.4f ms, fused pairs %.4f ms\n", dt,
              ms_mode[0] / 2, ms_mode[1] / 2);
  }
  g_timing = was_timing;
  drop_graphs(A);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // leave Y = A X computed with the tuned shapes
  s = qtt_apply(A, compute, nrhs, X, ldx, Y, ldy, ws, ws_bytes, stream);
  if (s != QTT_OK) return s;
  HIP_TRY(hipStreamSynchronize(st));
  return QTT_OK;
}

qtt_status_t qtt_list_shapes(qtt_dtype_t compute, int32_t* ids, int32_t cap, int32_t* count) {
  const int dt = dt_index(compute);
  if (dt < 0 || !count || (cap > 0 && !ids)) return fail(QTT_ERR_INVALID_ARG, "bad arguments");
  std::vector<int> v = shape_ids(dt, dt == 0);
  v.push_back(kSmallK);
  if (dt == 2) {
    v.push_back(kBf16Resident);
    v.push_back(kBf16Dma);
    v.push_back(kBf16Dma32);
    v.push_back(kBf16Last);
  }
  if (dt == 1) v.push_back(kValu32);
  if (dt == 0)
    for (auto& vc : valu_registry()) v.push_back(vc.id);
  *count = (int32_t)v.size();
  for (int i = 0; i < (int)v.size() && i < cap; ++i) ids[i] = v[i];
  return QTT_OK;
}

qtt_status_t qtt_set_shape(qtt_matrix_t A, qtt_dtype_t compute, int32_t core, int32_t shape) {
  if (!valid_handle(A)) return fail(QTT_ERR_INVALID_ARG, "null handle");
  int dt;
  qtt_status_t s = check_dtype(A, compute, &dt);
  if (s != QTT_OK) return s;
  if (core == -2) {               // fused core pairs (FP64, FP32) on/off
    if (dt == 2 || (shape != 0 && shape != 1)) return fail(QTT_ERR_INVALID_ARG, "core -2 takes shape 0 or 1 (FP64, FP32)");
    (dt == 0 ? A->fp64_pair : A->fp32_pair) = (shape == 1);
    drop_graphs(A);
    return QTT_OK;
  }
  if (core < 0 || core >= A->d) return fail(QTT_ERR_INVALID_ARG, "core %d out of range", core);
  if (shape != -1 && !(dt == 1 && shape == kF32Split)) {
    int32_t ids[128], n = 0;
    qtt_list_shapes(compute, ids, 128, &n);
    bool found = false;
    for (int i = 0; i < n && i < 128; ++i) found = found || ids[i] == shape;
    if (!found) return fail(QTT_ERR_INVALID_ARG, "shape %d is not a configuration for dtype %d", shape, (int)compute);
  }
  A->core[core].tuned[dt] = shape;
  // a pinned configuration is what runs: fused pairs would bypass it
  if (dt == 0 && shape != -1) A->fp64_pair = false;
  if (dt == 1 && shape != -1) A->fp32_pair = false;
  drop_graphs(A);
  return QTT_OK;
}

// --------------------------------------------------------------------------- solve

static size_t solve_extra_bytes(const qtt_matrix_s* A, int64_t nrhs) {
  return align256((size_t)A->rows * nrhs * 8)                 // residual R
         + align256((size_t)nrhs * kNormBlocks * 8)            // norm partials
         + align256((size_t)nrhs * 8);                         // norms
}

qtt_status_t qtt_solve_workspace_bytes(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                       int64_t nrhs, size_t* bytes) {
  if (!valid_handle(A) || !valid_handle(Ainv) || !bytes) return fail(QTT_ERR_INVALID_ARG, "null handle or output");
  int dt;
  qtt_status_t s = check_dtype(Ainv, inv_compute, &dt);
  if (s != QTT_OK) return s;
  s = check_dtype(A, QTT_FP64, &dt);
  if (s != QTT_OK) return s;
  const int64_t k = std::max<int64_t>(nrhs, 1);
  size_t wa = 0, wi = 0;
  qtt_workspace_bytes(A, QTT_FP64, k, &wa);
  qtt_workspace_bytes(Ainv, inv_compute, k, &wi);
  *bytes = std::max(wa, wi) + solve_extra_bytes(A, k);
  return QTT_OK;
}

static qtt_status_t column_norms(const std::vector<const double*>& cols, const std::vector<int64_t>& lds_,
                                 int64_t N, double* partial, double* dnorm, std::vector<double>& host,
                                 hipStream_t st) {
  // one launch per kNormCols columns (each column is its own segment)
  const int ncol = (int)cols.size();
  host.assign(ncol, 0.0);
  for (int c0 = 0; c0 < ncol; c0 += kNormCols) {
    NormArgs na;
    memset(&na, 0, sizeof(na));
    const int nc = std::min(kNormCols, ncol - c0);
    for (int t = 0; t < nc; ++t) {
      na.R[t] = cols[c0 + t];
      na.ld[t] = lds_[c0 + t];
      na.col_begin[t] = t;
    }
    na.nseg = nc;
    na.ncol = nc;
    na.N = N;
    na.partial = partial;
    void* args[] = {&na};
    HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&colnorm_partial_kernel), dim3(kNormBlocks, nc),
                            dim3(kNormThreads), args, 0, st));
    const double* pp = partial;
    int ncv = nc;
    double* dn = dnorm;
    void* args2[] = {&pp, &ncv, &dn};
    HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&colnorm_final_kernel), dim3((nc + 63) / 64), dim3(64),
                            args2, 0, st));
    HIP_TRY(hipMemcpyAsync(host.data() + c0, dnorm, nc * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  return QTT_OK;
}

// Checks of a solve's schedule against A (NULL sched: qtt_solve's).
static qtt_status_t check_schedule(const qtt_matrix_s* A, const qtt_schedule_t* sc, int* dt1, int* dtl) {
  if (!sc) return QTT_OK;
  if (sc->first_passes < 0) return fail(QTT_ERR_INVALID_ARG, "first_passes < 0");
  if (!(sc->lo_below >= 0) || !std::isfinite(sc->lo_below))
    return fail(QTT_ERR_INVALID_ARG, "lo_below must be finite and >= 0");
  qtt_status_t s;
  if (sc->first_passes > 0) {
    if (!valid_handle(sc->inv_first)) return fail(QTT_ERR_INVALID_ARG, "null inv_first with first_passes > 0");
    s = check_dtype(sc->inv_first, sc->first_compute, dt1);
    if (s != QTT_OK) return s;
  }
  if (sc->A_lo) {
    if (!valid_handle(sc->A_lo)) return fail(QTT_ERR_INVALID_ARG, "invalid A_lo");
    s = check_dtype(sc->A_lo, sc->lo_compute, dtl);
    if (s != QTT_OK) return s;
  }
  for (const qtt_matrix_s* M : {sc->first_passes > 0 ? sc->inv_first : nullptr, sc->A_lo}) {
    if (!M) continue;
    if (A->d != M->d) return fail(QTT_ERR_SHAPE, "schedule handle with a different core count");
    for (int k = 0; k < A->d; ++k)
      if (M->m[k] != A->m[k] || M->n[k] != A->n[k])
        return fail(QTT_ERR_SHAPE, "schedule handle with different modes (core %d)", k);
  }
  return QTT_OK;
}

// Apply workspace (per vector) of every handle a solve uses, and the bytes
// of the correction block.
static size_t schedule_apply_bytes(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                   const qtt_schedule_t* sc, int64_t k) {
  size_t need = 0, tmp = 0;
  qtt_workspace_bytes(A, QTT_FP64, k, &need);
  qtt_workspace_bytes(Ainv, inv_compute, k, &tmp);
  need = std::max(need, tmp);
  if (sc && sc->first_passes > 0) {
    qtt_workspace_bytes(sc->inv_first, sc->first_compute, k, &tmp);
    need = std::max(need, tmp);
  }
  if (sc && sc->A_lo) {
    qtt_workspace_bytes(sc->A_lo, sc->lo_compute, k, &tmp);
    need = std::max(need, tmp);
  }
  return need;
}

static size_t correction_bytes(const qtt_matrix_s* A, const qtt_schedule_t* sc, int64_t nrhs) {
  return (sc && sc->A_lo) ? align256((size_t)A->rows * nrhs * 8) : 0;
}

// y_c += x_c for the columns of each block (one launch per block).
static qtt_status_t add_cols(const std::vector<Block>& blocks, int64_t N, hipStream_t st) {
  for (const Block& b : blocks) {
    AddColsArgs aa;
    aa.y = b.y;
    aa.x = b.x;
    aa.ldy = b.ldy;
    aa.ldx = b.ldx;
    aa.N = N;
    const int64_t bx = std::min<int64_t>(1024, (N + 255) / 256);
    void* args[] = {&aa};
    HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&add_cols_kernel), dim3((unsigned)bx, (unsigned)b.width),
                            dim3(256), args, 0, st));
  }
  return QTT_OK;
}

// The refined solve with an optional schedule (NULL: qtt_solve).
static qtt_status_t solve_impl(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute, const qtt_schedule_t* sc,
                               int64_t nrhs, const double* F, int64_t ldf, double* Sigma, int64_t lds, double rtol,
                               int32_t max_iter, void* ws, size_t ws_bytes, void* stream, qtt_solve_col_t* info) {
  if (!valid_handle(A) || !valid_handle(Ainv)) return fail(QTT_ERR_INVALID_ARG, "null handle");
  int dti, dta, dt1 = -1, dtl = -1;
  qtt_status_t s = check_dtype(Ainv, inv_compute, &dti);
  if (s != QTT_OK) return s;
  s = check_dtype(A, QTT_FP64, &dta);
  if (s != QTT_OK) return s;
  if (A->d != Ainv->d) return fail(QTT_ERR_SHAPE, "A and Ainv have different core counts");
  for (int k = 0; k < A->d; ++k)
    if (A->m[k] != A->n[k] || Ainv->m[k] != A->m[k] || Ainv->n[k] != A->n[k])
      return fail(QTT_ERR_SHAPE, "solve needs square, identical modes (core %d)", k);
  s = check_schedule(A, sc, &dt1, &dtl);
  if (s != QTT_OK) return s;
  const int32_t first_passes = sc ? sc->first_passes : 0;
  const qtt_matrix_s* A_lo = sc ? sc->A_lo : nullptr;
  if (nrhs < 0 || max_iter < 1 || !(rtol >= 0)) return fail(QTT_ERR_INVALID_ARG, "bad nrhs, max_iter or rtol");
  if (nrhs == 0) return QTT_OK;
  if (!F || !Sigma || !ws) return fail(QTT_ERR_INVALID_ARG, "null F, Sigma or workspace");
  const int64_t N = A->rows;
  if (ldf < N || lds < N) return fail(QTT_ERR_INVALID_ARG, "ldf or lds < N");
  const size_t fb = ((size_t)(nrhs - 1) * ldf + N) * 8, sb = ((size_t)(nrhs - 1) * lds + N) * 8;
  if (overlaps(F, fb, Sigma, sb)) return fail(QTT_ERR_INVALID_ARG, "F and Sigma overlap");
  // carve the workspace: [R | D (with A_lo) | partial | norms | apply workspace]
  const size_t dbytes = correction_bytes(A, sc, nrhs);
  const size_t extra = solve_extra_bytes(A, nrhs) + dbytes;
  const size_t need1 = schedule_apply_bytes(A, Ainv, inv_compute, sc, 1);
  if (ws_bytes < extra + need1)
    return fail(QTT_ERR_WORKSPACE, "solve workspace %zu < minimum %zu", ws_bytes, extra + need1);
  if (overlaps(ws, ws_bytes, F, fb) || overlaps(ws, ws_bytes, Sigma, sb))
    return fail(QTT_ERR_INVALID_ARG, "workspace overlaps F or Sigma");
  char* p = static_cast<char*>(ws);
  double* R = reinterpret_cast<double*>(p);
  p += align256((size_t)N * nrhs * 8);
  double* D = dbytes ? reinterpret_cast<double*>(p) : nullptr;
  p += dbytes;
  double* partial = reinterpret_cast<double*>(p);
  p += align256((size_t)nrhs * kNormBlocks * 8);
  double* dnorm = reinterpret_cast<double*>(p);
  p += align256((size_t)nrhs * 8);
  void* aws = p;
  const size_t aws_bytes = ws_bytes - extra;
  hipStream_t st = static_cast<hipStream_t>(stream);

  std::vector<const double*> fcols(nrhs);
  std::vector<int64_t> fld(nrhs, ldf);
  for (int64_t c = 0; c < nrhs; ++c) fcols[c] = F + c * ldf;
  std::vector<double> fn, rn;
  s = column_norms(fcols, fld, N, partial, dnorm, fn, st);
  if (s != QTT_OK) return s;
  // columns still iterating; a converged column is frozen, and so is a column
  // whose F or residual is not finite (the others go on: columns never mix)
  std::vector<char> active(nrhs, 1);
  std::vector<double> rel(nrhs, 1.0);          // relative residual before the next pass
  int64_t n_active = nrhs;
  int64_t first_bad = -1;
  for (int64_t c = 0; c < nrhs; ++c) {
    if (info) { info[c].iters = 0; info[c].rel_residual = (fn[c] > 0) ? 1.0 : 0.0; }
    if (!(fn[c] > 0)) rel[c] = 0.0;
    if (!std::isfinite(fn[c])) {
      if (info) info[c].rel_residual = fn[c];
      if (first_bad < 0) first_bad = c;
      active[c] = 0;
      --n_active;
    }
  }
  for (int it = 1; it <= max_iter && n_active > 0; ++it) {
    // runs of consecutive active columns with the same residual route: a
    // column that starts the pass at or below lo_below updates its residual
    // with A_lo (decided per column, so a column's arithmetic does not
    // depend on the other columns of the call)
    auto lo_col = [&](int64_t c) { return A_lo != nullptr && rel[c] <= sc->lo_below; };
    std::vector<std::pair<int64_t, int64_t>> runs;
    for (int64_t c = 0; c < nrhs;) {
      if (!active[c]) { ++c; continue; }
      int64_t e = c;
      while (e < nrhs && active[e] && lo_col(e) == lo_col(c)) ++e;
      runs.push_back({c, e - c});
      c = e;
    }
    const bool use_first = it <= first_passes;
    const qtt_matrix_s* Ai = use_first ? sc->inv_first : Ainv;
    const int dtv = use_first ? dt1 : dti;
    std::vector<Block> bi, ba, bl, bd;
    for (auto& r : runs) {
      const int64_t c0 = r.first, w = r.second;
      if (!lo_col(c0)) {
        // sigma += Ainv r  (first pass: sigma = Ainv F); r = F - A sigma,
        // the residual fused into A's last core
        if (it == 1) bi.push_back({F + c0 * ldf, Sigma + c0 * lds, nullptr, ldf, lds, 0, w});
        else bi.push_back({R + c0 * N, Sigma + c0 * lds, Sigma + c0 * lds, N, lds, lds, w});
        ba.push_back({Sigma + c0 * lds, R + c0 * N, F + c0 * ldf, lds, N, ldf, w});
      } else if (it == 1) {
        // sigma = dx = Ainv F; r = F - A_lo sigma
        bi.push_back({F + c0 * ldf, Sigma + c0 * lds, nullptr, ldf, lds, 0, w});
        bl.push_back({Sigma + c0 * lds, R + c0 * N, F + c0 * ldf, lds, N, ldf, w});
      } else {
        // dx = Ainv r; sigma += dx; r -= A_lo dx
        bi.push_back({R + c0 * N, D + c0 * N, nullptr, N, N, 0, w});
        bd.push_back({D + c0 * N, Sigma + c0 * lds, nullptr, N, lds, 0, w});
        bl.push_back({D + c0 * N, R + c0 * N, R + c0 * N, N, N, N, w});
      }
    }
    s = run_blocks(Ai, dtv, bi, aws, aws_bytes, 1.0, st);
    if (s != QTT_OK) return s;
    if (!bd.empty()) {
      s = add_cols(bd, N, st);
      if (s != QTT_OK) return s;
    }
    s = run_blocks(A, dta, ba, aws, aws_bytes, -1.0, st);          // no-op without blocks
    if (s != QTT_OK) return s;
    if (!bl.empty()) {
      s = run_blocks(A_lo, dtl, bl, aws, aws_bytes, -1.0, st);
      if (s != QTT_OK) return s;
    }
    std::vector<const double*> rc;
    std::vector<int64_t> rld;
    std::vector<int64_t> idx;
    for (int64_t c = 0; c < nrhs; ++c)
      if (active[c]) { rc.push_back(R + c * N); rld.push_back(N); idx.push_back(c); }
    s = column_norms(rc, rld, N, partial, dnorm, rn, st);
    if (s != QTT_OK) return s;
    for (size_t t = 0; t < idx.size(); ++t) {
      const int64_t c = idx[t];
      const double rr = (fn[c] > 0) ? rn[t] / fn[c] : rn[t];
      rel[c] = rr;
      if (info) { info[c].iters = it; info[c].rel_residual = rr; }
      if (!std::isfinite(rr)) {
        if (first_bad < 0) first_bad = c;
        active[c] = 0;
        --n_active;
        continue;
      }
      if (rr <= rtol) { active[c] = 0; --n_active; }
    }
  }
  if (first_bad >= 0)
    return fail(QTT_ERR_NONFINITE, "column %lld: F or its residual is not finite", (long long)first_bad);
  if (n_active > 0) return fail(QTT_ERR_NOT_CONVERGED, "%lld columns above rtol after %d passes", (long long)n_active, max_iter);
  return QTT_OK;
}

qtt_status_t qtt_solve(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute, int64_t nrhs,
                       const double* F, int64_t ldf, double* Sigma, int64_t lds, double rtol,
                       int32_t max_iter, void* ws, size_t ws_bytes, void* stream, qtt_solve_col_t* info) {
  return solve_impl(A, Ainv, inv_compute, nullptr, nrhs, F, ldf, Sigma, lds, rtol, max_iter, ws, ws_bytes, stream,
                    info);
}

qtt_status_t qtt_solve_schedule_workspace_bytes(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                                const qtt_schedule_t* sched, int64_t nrhs, size_t* bytes) {
  if (!valid_handle(A) || !valid_handle(Ainv) || !bytes) return fail(QTT_ERR_INVALID_ARG, "null handle or output");
  int dt, dt1, dtl;
  qtt_status_t s = check_dtype(Ainv, inv_compute, &dt);
  if (s != QTT_OK) return s;
  s = check_dtype(A, QTT_FP64, &dt);
  if (s != QTT_OK) return s;
  s = check_schedule(A, sched, &dt1, &dtl);
  if (s != QTT_OK) return s;
  const int64_t k = std::max<int64_t>(nrhs, 1);
  *bytes = schedule_apply_bytes(A, Ainv, inv_compute, sched, k) + solve_extra_bytes(A, k) +
           correction_bytes(A, sched, k);
  return QTT_OK;
}

qtt_status_t qtt_solve_schedule(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                const qtt_schedule_t* sched, int64_t nrhs, const double* F, int64_t ldf,
                                double* Sigma, int64_t lds, double rtol, int32_t max_iter, void* ws,
                                size_t ws_bytes, void* stream, qtt_solve_col_t* info) {
  return solve_impl(A, Ainv, inv_compute, sched, nrhs, F, ldf, Sigma, lds, rtol, max_iter, ws, ws_bytes, stream,
                    info);
}

// --------------------------------------------------------------------------- flexible GMRES

// [V: max_iter + 1 blocks | Z: max_iter blocks (with a preconditioner) |
//  Gram partials | h1 | h2 | coefficients | norm partials | norms | apply ws]
// where a block is N x nrhs FP64 and the small buffers are sized per chunk
// of kKryCols columns.
static size_t fgmres_extra_bytes(const qtt_matrix_s* A, bool precond, int64_t nrhs, int32_t max_iter) {
  const size_t blk = align256((size_t)A->rows * nrhs * 8);
  // one chunk more than the columns need: finished and continuing columns
  // are chunked separately within a step
  const int64_t chunks = (nrhs + kKryCols - 1) / kKryCols + 1;
  const size_t hsz = align256((size_t)chunks * (max_iter + 1) * kKryCols * 8);
  return blk * (max_iter + 1) + (precond ? blk * max_iter : 0)
         + align256((size_t)kGramNb * kKryCols * kGramBlocks * 8)
         + 3 * hsz
         + align256((size_t)nrhs * kNormBlocks * 8) + align256((size_t)nrhs * 8);
}

qtt_status_t qtt_fgmres_workspace_bytes(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                        int64_t nrhs, int32_t max_iter, size_t* bytes) {
  if (!valid_handle(A) || (Ainv && !valid_handle(Ainv)) || !bytes)
    return fail(QTT_ERR_INVALID_ARG, "null handle or output");
  if (max_iter < 1) return fail(QTT_ERR_INVALID_ARG, "max_iter < 1");
  int dt;
  qtt_status_t s = check_dtype(A, QTT_FP64, &dt);
  if (s != QTT_OK) return s;
  const int64_t k = std::max<int64_t>(nrhs, 1);
  size_t wa = 0, wi = 0;
  qtt_workspace_bytes(A, QTT_FP64, k, &wa);
  if (Ainv) {
    s = check_dtype(Ainv, inv_compute, &dt);
    if (s != QTT_OK) return s;
    qtt_workspace_bytes(Ainv, inv_compute, k, &wi);
  }
  *bytes = std::max(wa, wi) + fgmres_extra_bytes(A, Ainv != nullptr, k, max_iter);
  return QTT_OK;
}

}  // extern "C"

namespace {

// One launch group of at most kKryCols columns.
struct KryChunk {
  int ncol = 0;
  int32_t col[kKryCols];
};

std::vector<KryChunk> chunk_columns(const std::vector<int64_t>& cols) {
  std::vector<KryChunk> out;
  for (size_t t = 0; t < cols.size(); t += kKryCols) {
    KryChunk ch;
    ch.ncol = (int)std::min<size_t>(kKryCols, cols.size() - t);
    for (int q = 0; q < ch.ncol; ++q) ch.col[q] = (int32_t)cols[t + q];
    out.push_back(ch);
  }
  return out;
}

// h[i * ncol + s] = <basis_i, w> for i < nb, columns of one chunk
qtt_status_t gram(const KryChunk& ch, const double* basis, int64_t bstride, int nb, const double* w,
                  int64_t N, double* partial, double* h, hipStream_t st) {
  for (int i0 = 0; i0 < nb; i0 += kGramNb) {
    GramArgs ga;
    memset(&ga, 0, sizeof(ga));
    ga.basis = basis + i0 * bstride;
    ga.bstride = bstride;
    ga.w = w;
    ga.N = N;
    ga.nb = std::min(kGramNb, nb - i0);
    ga.ncol = ch.ncol;
    memcpy(ga.col, ch.col, sizeof(ga.col));
    ga.partial = partial;
    void* args[] = {&ga};
    HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&gram_partial_kernel), dim3(kGramBlocks, ch.ncol),
                            dim3(kKryThreads), args, 0, st));
    const double* pp = partial;
    int nbv = ga.nb, nc = ch.ncol, i0v = i0;
    double* hv = h;
    void* args2[] = {&pp, &nbv, &nc, &i0v, &hv};
    const int nt = nbv * nc;
    HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&gram_final_kernel), dim3((nt + 63) / 64), dim3(64),
                            args2, 0, st));
  }
  return QTT_OK;
}

// out = scale * in + sign * sum_i coef_i basis_i, columns of one chunk
qtt_status_t combine(const KryChunk& ch, double* out, int64_t ldo, const double* in, int64_t ldi,
                     const double* scale, const double* basis, int64_t bstride, const double* coef, int nb,
                     double sign, int64_t N, hipStream_t st) {
  CombineArgs ca;
  memset(&ca, 0, sizeof(ca));
  ca.out = out;
  ca.ldo = ldo;
  ca.in = in;
  ca.ldi = ldi;
  ca.scale = scale;
  ca.basis = basis;
  ca.bstride = bstride;
  ca.coef = coef;
  ca.sign = sign;
  ca.N = N;
  ca.nb = nb;
  ca.ncol = ch.ncol;
  memcpy(ca.col, ch.col, sizeof(ca.col));
  const int64_t bx = std::min<int64_t>(512, std::max<int64_t>(1, (N + kKryThreads - 1) / kKryThreads));
  void* args[] = {&ca};
  HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&combine_kernel), dim3((unsigned)bx, ch.ncol),
                          dim3(kKryThreads), args, 0, st));
  return QTT_OK;
}

}  // namespace

extern "C" {

// Flexible GMRES with the preconditioner z = Ainv (Y v) (Y may be NULL: z =
// Ainv v; Ainv NULL: z = v).
static qtt_status_t fgmres_impl(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_matrix_t Y, qtt_dtype_t inv_compute,
                                int64_t nrhs, const double* F, int64_t ldf, double* Sigma, int64_t lds,
                                double rtol, int32_t max_iter, void* ws, size_t ws_bytes, void* stream,
                                qtt_solve_col_t* info, const qtt_schedule_t* sc = nullptr) {
  if (!valid_handle(A) || (Ainv && !valid_handle(Ainv)) || (Y && !valid_handle(Y)))
    return fail(QTT_ERR_INVALID_ARG, "null handle");
  int dti = -1, dta, dt1 = -1, dtl = -1;
  qtt_status_t s = check_dtype(A, QTT_FP64, &dta);
  if (s != QTT_OK) return s;
  s = check_schedule(A, sc, &dt1, &dtl);
  if (s != QTT_OK) return s;
  if (sc && sc->first_passes > 0 && !Ainv)
    return fail(QTT_ERR_INVALID_ARG, "first_passes > 0 needs a preconditioner");
  const qtt_matrix_s* A_lo = sc ? sc->A_lo : nullptr;
  for (qtt_matrix_t P : {Ainv, Y}) {
    if (!P) continue;
    s = check_dtype(P, inv_compute, &dti);
    if (s != QTT_OK) return s;
    if (A->d != P->d) return fail(QTT_ERR_SHAPE, "A and the preconditioner have different core counts");
    for (int k = 0; k < A->d; ++k)
      if (P->m[k] != A->m[k] || P->n[k] != A->n[k])
        return fail(QTT_ERR_SHAPE, "solve needs square, identical modes (core %d)", k);
  }
  for (int k = 0; k < A->d; ++k)
    if (A->m[k] != A->n[k]) return fail(QTT_ERR_SHAPE, "solve needs square, identical modes (core %d)", k);
  if (nrhs < 0 || max_iter < 1 || !(rtol >= 0)) return fail(QTT_ERR_INVALID_ARG, "bad nrhs, max_iter or rtol");
  if (nrhs == 0) return QTT_OK;
  if (!F || !Sigma || !ws) return fail(QTT_ERR_INVALID_ARG, "null F, Sigma or workspace");
  const int64_t N = A->rows;
  if (ldf < N || lds < N) return fail(QTT_ERR_INVALID_ARG, "ldf or lds < N");
  const size_t fb = ((size_t)(nrhs - 1) * ldf + N) * 8, sb = ((size_t)(nrhs - 1) * lds + N) * 8;
  if (overlaps(F, fb, Sigma, sb)) return fail(QTT_ERR_INVALID_ARG, "F and Sigma overlap");
  const bool pre = Ainv != nullptr;
  const size_t extra = fgmres_extra_bytes(A, pre, nrhs, max_iter);
  size_t need1 = 0, tmp = 0;
  qtt_workspace_bytes(A, QTT_FP64, 1, &need1);
  for (qtt_matrix_t P : {Ainv, Y}) {
    if (!P) continue;
    qtt_workspace_bytes(P, inv_compute, 1, &tmp);
    need1 = std::max(need1, tmp);
  }
  if (sc && sc->first_passes > 0) {
    qtt_workspace_bytes(sc->inv_first, sc->first_compute, 1, &tmp);
    need1 = std::max(need1, tmp);
  }
  if (A_lo) {
    qtt_workspace_bytes(sc->A_lo, sc->lo_compute, 1, &tmp);
    need1 = std::max(need1, tmp);
  }
  if (ws_bytes < extra + need1)
    return fail(QTT_ERR_WORKSPACE, "FGMRES workspace %zu < minimum %zu", ws_bytes, extra + need1);
  if (overlaps(ws, ws_bytes, F, fb) || overlaps(ws, ws_bytes, Sigma, sb))
    return fail(QTT_ERR_INVALID_ARG, "workspace overlaps F or Sigma");

  // carve the workspace
  const int64_t bstride = N * nrhs;   // one block: N x nrhs, column c at + c * N
  const size_t blk = align256((size_t)bstride * 8);
  const int64_t nchunk = (nrhs + kKryCols - 1) / kKryCols + 1;
  const int64_t hstride = (int64_t)(max_iter + 1) * kKryCols;   // per chunk
  const size_t hsz = align256((size_t)nchunk * hstride * 8);
  char* p = static_cast<char*>(ws);
  double* V = reinterpret_cast<double*>(p);
  p += blk * (max_iter + 1);
  double* Z = V;   // no preconditioner: z_j = v_j
  if (pre) {
    Z = reinterpret_cast<double*>(p);
    p += blk * max_iter;
  }
  double* gpart = reinterpret_cast<double*>(p);
  p += align256((size_t)kGramNb * kKryCols * kGramBlocks * 8);
  double* h1 = reinterpret_cast<double*>(p);
  p += hsz;
  double* h2 = reinterpret_cast<double*>(p);
  p += hsz;
  double* cbuf = reinterpret_cast<double*>(p);
  p += hsz;
  double* npart = reinterpret_cast<double*>(p);
  p += align256((size_t)nrhs * kNormBlocks * 8);
  double* dnorm = reinterpret_cast<double*>(p);
  p += align256((size_t)nrhs * 8);
  void* aws = p;
  const size_t aws_bytes = ws_bytes - extra;
  hipStream_t st = static_cast<hipStream_t>(stream);

  // ||f_c||
  std::vector<const double*> fcols(nrhs);
  std::vector<int64_t> fld(nrhs, ldf);
  for (int64_t c = 0; c < nrhs; ++c) fcols[c] = F + c * ldf;
  std::vector<double> beta;
  s = column_norms(fcols, fld, N, npart, dnorm, beta, st);
  if (s != QTT_OK) return s;
  std::vector<int64_t> act, zero;
  std::vector<double> relv(nrhs, 0.0);
  std::vector<double> est(nrhs, 1.0);     // residual estimate before the next step (A_lo routing)
  int64_t first_bad = -1;   // columns whose F is not finite are skipped (Sigma not written)
  for (int64_t c = 0; c < nrhs; ++c) {
    if (info) { info[c].iters = 0; info[c].rel_residual = 0.0; }
    if (!std::isfinite(beta[c])) {
      if (info) info[c].rel_residual = beta[c];
      if (first_bad < 0) first_bad = c;
      continue;
    }
    (beta[c] > 0 ? act : zero).push_back(c);
  }
  // zero right-hand sides: sigma = 0
  for (auto& ch : chunk_columns(zero)) {
    s = combine(ch, Sigma, lds, nullptr, 0, nullptr, nullptr, 0, nullptr, 0, 1.0, N, st);
    if (s != QTT_OK) return s;
  }
  // host state per column: Hessenberg columns (rotated), rotations, g
  const int M = max_iter;
  std::vector<double> H((size_t)nrhs * (M + 1) * M, 0.0), cs((size_t)nrhs * M), sn((size_t)nrhs * M),
      g((size_t)nrhs * (M + 1), 0.0);
  auto Hc = [&](int64_t c, int i, int j) -> double& { return H[((size_t)c * M + j) * (M + 1) + i]; };
  for (int64_t c : act) g[(size_t)c * (M + 1)] = beta[c];
  // host staging of uploaded coefficients: one region per chunk and purpose,
  // untouched until the stream has synchronised again
  std::vector<double> hscale((size_t)nchunk * hstride), hy((size_t)nchunk * hstride);
  std::vector<double> hh1((size_t)nchunk * hstride), hh2((size_t)nchunk * hstride);

  // v_1 = f / ||f||
  {
    auto chs = chunk_columns(act);
    for (size_t q = 0; q < chs.size(); ++q) {
      for (int t = 0; t < chs[q].ncol; ++t) hscale[q * hstride + t] = 1.0 / beta[chs[q].col[t]];
      HIP_TRY(hipMemcpyAsync(cbuf + q * hstride, hscale.data() + q * hstride, chs[q].ncol * 8,
                             hipMemcpyHostToDevice, st));
      // F columns are at F + c * ldf; V columns at V + c * N
      s = combine(chs[q], V, N, F, ldf, cbuf + q * hstride, nullptr, 0, nullptr, 0, 1.0, N, st);
      if (s != QTT_OK) return s;
    }
  }

  // x = Z y for the columns of one chunk after k steps (y solved on the host)
  auto finish = [&](const std::vector<int64_t>& cols, int k, size_t slot) -> qtt_status_t {
    auto chs = chunk_columns(cols);
    for (size_t q = 0; q < chs.size(); ++q) {
      double* hyq = hy.data() + (slot + q) * hstride;
      for (int t = 0; t < chs[q].ncol; ++t) {
        const int64_t c = chs[q].col[t];
        std::vector<double> y(k);
        for (int i = k - 1; i >= 0; --i) {
          double v = g[(size_t)c * (M + 1) + i];
          for (int l = i + 1; l < k; ++l) v -= Hc(c, i, l) * y[l];
          y[i] = v / Hc(c, i, i);
        }
        for (int i = 0; i < k; ++i) hyq[(size_t)i * chs[q].ncol + t] = y[i];
      }
      double* dy = cbuf + (slot + q) * hstride;
      HIP_TRY(hipMemcpyAsync(dy, hyq, (size_t)k * chs[q].ncol * 8, hipMemcpyHostToDevice, st));
      qtt_status_t r = combine(chs[q], Sigma, lds, nullptr, 0, nullptr, Z, bstride, dy, k, 1.0, N, st);
      if (r != QTT_OK) return r;
    }
    return QTT_OK;
  };

  for (int j = 0; j < M && !act.empty(); ++j) {
    // z_j = Ainv v_j, w = A z_j (w is stored as v_{j+1}); a column whose
    // residual estimate is at or below the schedule's lo_below forms
    // w = A_lo z_j (decided per column)
    auto lo_col = [&](int64_t c) { return A_lo != nullptr && est[c] <= sc->lo_below; };
    std::vector<std::pair<int64_t, int64_t>> runs;
    for (size_t t = 0; t < act.size();) {
      size_t e = t + 1;
      while (e < act.size() && act[e] == act[e - 1] + 1 && lo_col(act[e]) == lo_col(act[t])) ++e;
      runs.push_back({act[t], (int64_t)(e - t)});
      t = e;
    }
    double* Vj = V + j * bstride;
    double* Zj = Z + j * bstride;
    double* W = V + (j + 1) * bstride;
    std::vector<Block> bi, ba, bl, by;
    for (auto& r : runs) {
      // with a product preconditioner, Y v_j goes to the w slot first (A z_j
      // overwrites it afterwards)
      by.push_back({Vj + r.first * N, W + r.first * N, nullptr, N, N, 0, r.second});
      bi.push_back({(Y ? W : Vj) + r.first * N, Zj + r.first * N, nullptr, N, N, 0, r.second});
      (lo_col(r.first) ? bl : ba).push_back({Zj + r.first * N, W + r.first * N, nullptr, N, N, 0, r.second});
    }
    if (Y) {
      s = run_blocks(Y, dti, by, aws, aws_bytes, 1.0, st);
      if (s != QTT_OK) return s;
    }
    if (pre) {
      const bool first = sc && j < sc->first_passes;
      s = first ? run_blocks(sc->inv_first, dt1, bi, aws, aws_bytes, 1.0, st)
                : run_blocks(Ainv, dti, bi, aws, aws_bytes, 1.0, st);
      if (s != QTT_OK) return s;
    }
    s = run_blocks(A, dta, ba, aws, aws_bytes, 1.0, st);          // no-op without blocks
    if (s != QTT_OK) return s;
    if (!bl.empty()) {
      s = run_blocks(A_lo, dtl, bl, aws, aws_bytes, 1.0, st);
      if (s != QTT_OK) return s;
    }
    // classical Gram-Schmidt, twice: h = V^T w, w -= V h
    const int nb = j + 1;
    auto chs = chunk_columns(act);
    for (size_t q = 0; q < chs.size(); ++q) {
      double* hq1 = h1 + q * hstride;
      double* hq2 = h2 + q * hstride;
      s = gram(chs[q], V, bstride, nb, W, N, gpart, hq1, st);
      if (s != QTT_OK) return s;
      s = combine(chs[q], W, N, W, N, nullptr, V, bstride, hq1, nb, -1.0, N, st);
      if (s != QTT_OK) return s;
      s = gram(chs[q], V, bstride, nb, W, N, gpart, hq2, st);
      if (s != QTT_OK) return s;
      s = combine(chs[q], W, N, W, N, nullptr, V, bstride, hq2, nb, -1.0, N, st);
      if (s != QTT_OK) return s;
      HIP_TRY(hipMemcpyAsync(hh1.data() + q * hstride, hq1, (size_t)nb * chs[q].ncol * 8, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(hh2.data() + q * hstride, hq2, (size_t)nb * chs[q].ncol * 8, hipMemcpyDeviceToHost, st));
    }
    std::vector<const double*> wc;
    std::vector<int64_t> wld(act.size(), N);
    for (int64_t c : act) wc.push_back(W + c * N);
    std::vector<double> wn;
    s = column_norms(wc, wld, N, npart, dnorm, wn, st);   // synchronises the stream
    if (s != QTT_OK) return s;
    // Hessenberg column j, rotations, residual estimate
    std::vector<int64_t> done, keep;
    std::vector<double> keep_scale;
    for (size_t q = 0, t = 0; q < chs.size(); ++q) {
      for (int u = 0; u < chs[q].ncol; ++u, ++t) {
        const int64_t c = chs[q].col[u];
        for (int i = 0; i < nb; ++i)
          Hc(c, i, j) = hh1[q * hstride + (size_t)i * chs[q].ncol + u] + hh2[q * hstride + (size_t)i * chs[q].ncol + u];
        const double hn = wn[t];
        Hc(c, j + 1, j) = hn;
        double* cc = cs.data() + (size_t)c * M;
        double* ss = sn.data() + (size_t)c * M;
        for (int i = 0; i < j; ++i) {
          const double a = Hc(c, i, j), b = Hc(c, i + 1, j);
          Hc(c, i, j) = cc[i] * a + ss[i] * b;
          Hc(c, i + 1, j) = -ss[i] * a + cc[i] * b;
        }
        const double d = std::hypot(Hc(c, j, j), Hc(c, j + 1, j));
        if (!std::isfinite(d) || !std::isfinite(hn))
          return fail(QTT_ERR_NONFINITE, "Arnoldi step %d of column %lld is not finite", j + 1, (long long)c);
        if (d == 0.0) return fail(QTT_ERR_NONFINITE, "singular Hessenberg at step %d, column %lld", j + 1, (long long)c);
        cc[j] = Hc(c, j, j) / d;
        ss[j] = Hc(c, j + 1, j) / d;
        Hc(c, j, j) = d;
        Hc(c, j + 1, j) = 0.0;
        double* gc = g.data() + (size_t)c * (M + 1);
        gc[j + 1] = -ss[j] * gc[j];
        gc[j] = cc[j] * gc[j];
        const double rel = std::fabs(gc[j + 1]) / beta[c];
        relv[c] = rel;
        est[c] = rel;
        if (info) { info[c].iters = j + 1; info[c].rel_residual = rel; }
        if (rel <= rtol || hn == 0.0 || j + 1 == M) done.push_back(c);
        else { keep.push_back(c); keep_scale.push_back(1.0 / hn); }
      }
    }
    // finished columns: sigma = Z y now (their blocks are not touched again)
    if (!done.empty()) {
      s = finish(done, j + 1, 0);
      if (s != QTT_OK) return s;
    }
    // the others: v_{j+1} = w / h_{j+1,j}
    auto kch = chunk_columns(keep);
    const size_t off = chunk_columns(done).size();
    for (size_t q = 0, t = 0; q < kch.size(); ++q) {
      double* hs = hscale.data() + (off + q) * hstride;
      for (int u = 0; u < kch[q].ncol; ++u, ++t) hs[u] = keep_scale[t];
      double* ds = cbuf + (off + q) * hstride;
      HIP_TRY(hipMemcpyAsync(ds, hs, kch[q].ncol * 8, hipMemcpyHostToDevice, st));
      s = combine(kch[q], W, N, W, N, ds, nullptr, 0, nullptr, 0, 1.0, N, st);
      if (s != QTT_OK) return s;
    }
    act.swap(keep);
  }
  // every column is finished here (the last step finishes the rest)
  int64_t above = 0;
  for (int64_t c = 0; c < nrhs; ++c) above += (relv[c] > rtol);
  HIP_TRY(hipStreamSynchronize(st));
  if (first_bad >= 0) return fail(QTT_ERR_NONFINITE, "column %lld of F is not finite", (long long)first_bad);
  if (above > 0) return fail(QTT_ERR_NOT_CONVERGED, "%lld columns above rtol after %d steps", (long long)above, M);
  return QTT_OK;
}

qtt_status_t qtt_solve_fgmres(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute, int64_t nrhs,
                              const double* F, int64_t ldf, double* Sigma, int64_t lds, double rtol,
                              int32_t max_iter, void* ws, size_t ws_bytes, void* stream,
                              qtt_solve_col_t* info) {
  return fgmres_impl(A, Ainv, nullptr, inv_compute, nrhs, F, ldf, Sigma, lds, rtol, max_iter, ws, ws_bytes,
                     stream, info);
}

qtt_status_t qtt_fgmres_schedule_workspace_bytes(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                                 const qtt_schedule_t* sched, int64_t nrhs, int32_t max_iter,
                                                 size_t* bytes) {
  qtt_status_t s = qtt_fgmres_workspace_bytes(A, Ainv, inv_compute, nrhs, max_iter, bytes);
  if (s != QTT_OK) return s;
  int dt1, dtl;
  s = check_schedule(A, sched, &dt1, &dtl);
  if (s != QTT_OK) return s;
  if (!sched) return QTT_OK;
  const int64_t k = std::max<int64_t>(nrhs, 1);
  size_t wa = 0, tmp = 0;
  qtt_workspace_bytes(A, QTT_FP64, k, &wa);
  size_t wmax = wa;
  if (Ainv) {
    qtt_workspace_bytes(Ainv, inv_compute, k, &tmp);
    wmax = std::max(wmax, tmp);
  }
  size_t wsched = wmax;
  if (sched->first_passes > 0) {
    qtt_workspace_bytes(sched->inv_first, sched->first_compute, k, &tmp);
    wsched = std::max(wsched, tmp);
  }
  if (sched->A_lo) {
    qtt_workspace_bytes(sched->A_lo, sched->lo_compute, k, &tmp);
    wsched = std::max(wsched, tmp);
  }
  *bytes += wsched - wmax;
  return QTT_OK;
}

qtt_status_t qtt_solve_fgmres_schedule(qtt_matrix_t A, qtt_matrix_t Ainv, qtt_dtype_t inv_compute,
                                       const qtt_schedule_t* sched, int64_t nrhs, const double* F, int64_t ldf,
                                       double* Sigma, int64_t lds, double rtol, int32_t max_iter, void* ws,
                                       size_t ws_bytes, void* stream, qtt_solve_col_t* info) {
  return fgmres_impl(A, Ainv, nullptr, inv_compute, nrhs, F, ldf, Sigma, lds, rtol, max_iter, ws, ws_bytes,
                     stream, info, sched);
}

qtt_status_t qtt_solve_fgmres_product(qtt_matrix_t A, qtt_matrix_t M, qtt_matrix_t Y, qtt_dtype_t inv_compute,
                                      int64_t nrhs, const double* F, int64_t ldf, double* Sigma, int64_t lds,
                                      double rtol, int32_t max_iter, void* ws, size_t ws_bytes, void* stream,
                                      qtt_solve_col_t* info) {
  if (!M || !Y) return fail(QTT_ERR_INVALID_ARG, "the product preconditioner needs both M and Y");
  return fgmres_impl(A, M, Y, inv_compute, nrhs, F, ldf, Sigma, lds, rtol, max_iter, ws, ws_bytes, stream,
                     info);
}

// --------------------------------------------------------------------------- compressed product

qtt_status_t qtt_matvec_compressed(qtt_matrix_t A, int64_t nvec, const int64_t* rb, const double* const* B,
                                   double* const* C, void* stream) {
  if (!valid_handle(A)) return fail(QTT_ERR_INVALID_ARG, "null handle");
  int dt;
  qtt_status_t s = check_dtype(A, QTT_FP64, &dt);
  if (s != QTT_OK) return s;
  if (A->has_diag) return fail(QTT_ERR_INVALID_ARG, "an operator with diagonals has no compressed product here");
  if (nvec < 0) return fail(QTT_ERR_INVALID_ARG, "nvec < 0");
  if (nvec == 0) return QTT_OK;
  if (!rb || !B || !C) return fail(QTT_ERR_INVALID_ARG, "null rank or core array");
  const int d = A->d;
  if (rb[0] != 1 || rb[d] != 1) return fail(QTT_ERR_SHAPE, "vector ranks must start and end with 1");
  std::vector<std::pair<const void*, size_t>> ins, outs;
  for (int k = 0; k < d; ++k) {
    if (rb[k + 1] < 1 || rb[k + 1] * A->core[k].r_out > (1 << 24))
      return fail(QTT_ERR_SHAPE, "vector rank %d out of range", k + 1);
    if (!B[k] || !C[k]) return fail(QTT_ERR_INVALID_ARG, "core %d pointer is null", k);
    const CoreDev& c = A->core[k];
    const size_t ib = (size_t)nvec * rb[k] * c.n * rb[k + 1] * 8;
    const size_t ob = (size_t)nvec * rb[k] * c.r_in * c.m * rb[k + 1] * c.r_out * 8;
    ins.push_back({B[k], ib});
    outs.push_back({C[k], ob});
  }
  for (size_t i = 0; i < outs.size(); ++i) {
    for (auto& x : ins)
      if (overlaps(outs[i].first, outs[i].second, x.first, x.second)) return fail(QTT_ERR_INVALID_ARG, "output core %zu overlaps an input core", i);
    for (size_t j = 0; j < i; ++j)
      if (overlaps(outs[i].first, outs[i].second, outs[j].first, outs[j].second)) return fail(QTT_ERR_INVALID_ARG, "output cores %zu and %zu overlap", j, i);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int k = 0; k < d; ++k) {
    const CoreDev& c = A->core[k];
    CmvArgs ca;
    ca.G = c.g64;
    ca.B = B[k];
    ca.C = C[k];
    ca.nvec = nvec;
    ca.ra0 = c.r_in;
    ca.ra1 = c.r_out;
    ca.rb0 = (int32_t)rb[k];
    ca.rb1 = (int32_t)rb[k + 1];
    ca.m = c.m;
    ca.n = c.n;
    void* args[] = {&ca};
    if (c.n <= kCmvMaxN && c.n * rb[k + 1] <= kCmvLds && c.r_out <= 256) {
      const int64_t nchunk = ((int64_t)c.r_in * c.m + kCmvRows - 1) / kCmvRows;
      const int64_t blocks = std::min<int64_t>(1 << 18, std::max<int64_t>(1, nvec * rb[k] * nchunk));
      HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&compressed_matvec_lds_kernel),
                              dim3((unsigned)blocks), dim3(256), args, 0, st));
      continue;
    }
    const int64_t rows = (int64_t)nvec * rb[k] * c.r_in * c.m;
    const int64_t R = rb[k + 1] * c.r_out;
    const int64_t rpb = (R >= 256) ? 1 : 256 / R;
    const int64_t blocks = std::min<int64_t>(1 << 18, std::max<int64_t>(1, (rows + rpb - 1) / rpb));
    HIP_TRY(hipLaunchKernel(reinterpret_cast<const void*>(&compressed_matvec_kernel), dim3((unsigned)blocks),
                            dim3(256), args, 0, st));
  }
  return QTT_OK;
}

// --------------------------------------------------------------------------- timing

qtt_status_t qtt_timing_enable(int32_t on) {
  g_timing = on != 0;
  return QTT_OK;
}

qtt_status_t qtt_timing_reset(void) {
  for (auto& t : g_timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  g_timed.clear();
  return QTT_OK;
}

// launches of one dtype selected by core position (by_shape == false) or by
// kernel configuration id (by_shape == true)
static qtt_status_t timing_sum(int dt, bool by_shape, int key, int64_t* launches, double* milliseconds,
                               double* flops, double* bytes) {
  int64_t n = 0;
  double ms = 0, fl = 0, by = 0;
  for (auto& t : g_timed) {
    if (t.dt != dt || (by_shape ? t.shape : t.pos) != key) continue;
    HIP_TRY(hipEventSynchronize(t.b));
    float e = 0;
    HIP_TRY(hipEventElapsedTime(&e, t.a, t.b));
    ++n;
    ms += e;
    fl += t.flops;
    by += t.bytes;
  }
  if (launches) *launches = n;
  if (milliseconds) *milliseconds = ms;
  if (flops) *flops = fl;
  if (bytes) *bytes = by;
  return QTT_OK;
}

qtt_status_t qtt_timing_read(qtt_dtype_t compute, int32_t position, int64_t* launches, double* milliseconds,
                             double* flops, double* bytes) {
  const int dt = dt_index(compute);
  if (dt < 0 || position < 0 || position > 3) return fail(QTT_ERR_INVALID_ARG, "bad dtype or position");
  return timing_sum(dt, false, position, launches, milliseconds, flops, bytes);
}

qtt_status_t qtt_timing_read_shape(qtt_dtype_t compute, int32_t shape, int64_t* launches,
                                   double* milliseconds, double* flops, double* bytes) {
  const int dt = dt_index(compute);
  if (dt < 0) return fail(QTT_ERR_INVALID_ARG, "bad dtype");
  return timing_sum(dt, true, shape, launches, milliseconds, flops, bytes);
}

}  // extern "C"
