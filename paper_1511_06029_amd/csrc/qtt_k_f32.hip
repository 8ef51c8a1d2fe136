// FP32 core-step kernel configurations (packed FP32 input, and FP64 input for the first core),
// and the FP32 interior step formed from split BF16 products.
#define QTT_KERNEL_TEMPLATES_ONLY
#include "qtt_families.hpp"

namespace qtt {

void add_kernels_f32(std::vector<KernelCfg>& v) {
  add_family<float, float, 32, 32>(v, 1, false);
  add_family<float, double, 32, 32>(v, 1, true);
}

const void* f32_split_kernel(int spt) {
  switch (spt) {
    case 1: return reinterpret_cast<const void*>(&core_step_f32_split_kernel<1>);
    case 2: return reinterpret_cast<const void*>(&core_step_f32_split_kernel<2>);
    case 3: return reinterpret_cast<const void*>(&core_step_f32_split_kernel<3>);
    case 4: return reinterpret_cast<const void*>(&core_step_f32_split_kernel<4>);
    default: return nullptr;
  }
}

}  // namespace qtt
