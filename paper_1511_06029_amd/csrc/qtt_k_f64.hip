// FP64 core-step kernel configurations.
#define QTT_KERNEL_TEMPLATES_ONLY
#include "qtt_families.hpp"

namespace qtt {

void add_kernels_f64(std::vector<KernelCfg>& v) { add_family<double, double, 32, 16>(v, 0, true); }

}  // namespace qtt
