// FP32 core-step kernel configurations (packed FP32 input, and FP64 input for the first core).
#define QTT_KERNEL_TEMPLATES_ONLY
#include "qtt_families.hpp"

namespace qtt {

void add_kernels_f32(std::vector<KernelCfg>& v) {
  add_family<float, float, 32, 32>(v, 1, false);
  add_family<float, double, 32, 32>(v, 1, true);
}

}  // namespace qtt
