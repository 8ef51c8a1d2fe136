// BF16 core-step kernel configurations, the direct-to-LDS BF16 interior kernel
// and the register-streamed BF16 last core.
#define QTT_KERNEL_TEMPLATES_ONLY
#include "qtt_families.hpp"

namespace qtt {

void add_kernels_bf16(std::vector<KernelCfg>& v) {
  add_family<bf16_tag, uint16_t, 128, 64>(v, 2, false);
  add_family<bf16_tag, double, 32, 64>(v, 2, true);   // first core: K_in = n_1 is small
}

const void* bf16_last_kernel() { return reinterpret_cast<const void*>(&core_step_bf16_last_kernel<8>); }

const void* bf16_dma_kernel(int tcb) {
  return tcb == 2 ? reinterpret_cast<const void*>(&core_step_bf16_dma_kernel<2>)
                  : reinterpret_cast<const void*>(&core_step_bf16_dma_kernel<4>);
}

}  // namespace qtt
