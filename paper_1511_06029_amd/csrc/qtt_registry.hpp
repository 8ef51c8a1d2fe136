// Kernel tables of libqtt.  The kernel templates are instantiated in
// several translation units (one per dtype family, one for the fused pairs,
// one for the vector-ALU kernels) so that they compile in parallel; each
// unit exports its table through the functions declared here, and the
// runtime only ever sees kernel symbols as pointers.
#pragma once

#include <vector>

#include "qtt_kernels.hpp"

namespace qtt {

struct KernelCfg {
  int dt;          // 0 fp64, 1 fp32, 2 bf16
  bool in_f64;     // reads FP64 input (first core)
  bool vec;        // 16-byte input loads
  int TR, TC, KC, NT;
  int id;          // configuration id within the dtype (tile shape)
  const void* fn;  // kernel symbol
  int occ;         // resident blocks per CU, 0 = not yet queried
  int kind;        // 0 single-operand LDS, 2 streamed, 3 4x4x4 streamed
};

// FP64 vector-ALU kernels: (id, waves, rows per wave, columns per lane, input group size,
// groups loaded per step).
struct ValuCfg {
  int id, NW, RW, CPL, G, LG;
  const void* fn;
  int occ;
};

constexpr int kGenericShape = 6;   // scalar-load fallback of every family
constexpr int kSmallK = 34;        // first core with a short contraction (vector ALUs)
constexpr int kValuGeneric = 48;   // vector-ALU kernel without input groups

// matrix-core tile configurations per dtype (qtt_k_f64.hip, qtt_k_f32.hip, qtt_k_bf16.hip)
void add_kernels_f64(std::vector<KernelCfg>& v);
void add_kernels_f32(std::vector<KernelCfg>& v);
void add_kernels_bf16(std::vector<KernelCfg>& v);
// core_step_bf16_dma_kernel<tcb>, tcb = 2 or 4, and core_step_bf16_last_kernel (qtt_k_bf16.hip)
const void* bf16_dma_kernel(int tcb);
const void* bf16_last_kernel();
// core_step_f32_split_kernel<spt>: FP32 interior step from split BF16 products,
// R_out = 64 spt, spt = 1..4 (qtt_k_f32.hip)
const void* f32_split_kernel(int spt);
// fused core pairs (qtt_k_pair64.hip, qtt_k_pair32.hip); index
// 6 first + 2 (0: rank 24, 1: rank 32, 2: padded 17..32) + (rows of core k + 1 > 192)
const void* pair_f64_kernel(int f);
const void* pair_f32_kernel(int f);
// FP64 vector-ALU kernels and the short-contraction first core (qtt_k_misc.hip;
// smallk_kernel(3), smallk_kernel(4): the BF16 and FP32 first cores with rows
// in registers)
void add_valu_kernels(std::vector<ValuCfg>& v);
// the FP32 last core on the vector ALUs (core_step_valu32_kernel), id 39
ValuCfg valu32_last_cfg();
const void* smallk_kernel(int dt);

}  // namespace qtt
