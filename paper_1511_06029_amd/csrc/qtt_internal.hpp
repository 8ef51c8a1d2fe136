// Internal declarations shared by the host translation units of libqtt: the
// matrix handle, error reporting, and the HIP-call check.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "qtt.h"

namespace qtt {

// Record a message for qtt_last_error() on this thread and return s.
qtt_status_t fail(qtt_status_t s, const char* fmt, ...);

}  // namespace qtt

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return qtt::fail(QTT_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// the matrix handle
// ---------------------------------------------------------------------------
struct CoreDev {
  int r_in, r_out, m, n;
  int R_out, K_in;
  int64_t C;          // columns of b_k per vector
  int64_t out_len;    // elements of y_k per vector
  int nRB;
  int Ksteps[3];
  void* frag[3];
  int tuned[3];       // tuned shape id per dtype, -1 = heuristic
  double* valu;       // FP64 vector-ALU copy Mv, input groups of 8 (when K_in % 8 == 0)
  double* valu1;      // FP64 vector-ALU copy Mv, groups of 1
  float* valu32 = nullptr;  // FP32 vector-ALU copy Mv, groups of 8 (last core, K_in % 32 == 0)
  int Rpad;           // rows of Mv
  double* g64 = nullptr;  // FP64 core as given, [r_in][m][n][r_out] (compressed products)
  // FP32 core split into BF16 hi and lo fragment arrays (hi, then lo, each in
  // the BF16 fragment layout with fsplit_ks steps), for K_in <= 256, K_in % 8 == 0
  void* fsplit = nullptr;
  int fsplit_ks = 0;
  int32_t fsplit_half = 0;  // bytes of one of the two arrays
};

struct qtt_matrix_s {
  int d = 0;
  std::vector<int64_t> ranks, m, n;
  int64_t rows = 0, cols = 0, max_rank = 0;
  uint32_t dtypes = 0;
  int device = 0;
  std::vector<CoreDev> core;
  int64_t max_inter = 0;  // largest y_k (k < d) per vector, elements
  bool fp64_pair = true;  // FP64 sweeps fuse interior core pairs where the pair kernel applies
  bool fp32_pair = true;  // the same for FP32 sweeps
  // a I + diag(b) K diag(wc) (non-translation-invariant operator); device
  // arrays of rows / cols values, NULL = ones
  bool has_diag = false;
  double diag_a = 0.0;
  double* diag_b = nullptr;
  double* diag_wc = nullptr;
  // captured sweeps: a sweep with the same dtype, vectors, pointers, workspace
  // and alpha replays its graph instead of launching d kernels
  struct Graph {
    std::string key;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipEvent_t done;   // recorded after each launch: waited on before destruction
  };
  mutable std::mutex graph_mu;
  mutable std::vector<Graph> graphs;   // most recent last
  mutable hipStream_t cap_stream = nullptr;
  mutable uint64_t tune_gen = 0;       // bumped when tile choices change
};

