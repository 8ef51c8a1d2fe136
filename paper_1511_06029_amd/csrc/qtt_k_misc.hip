// FP64 vector-ALU core-step kernels, the FP32 vector-ALU last core and the
// short-contraction first-core kernels.
#define QTT_KERNEL_TEMPLATES_ONLY
#include "qtt_registry.hpp"

namespace qtt {

// (id, waves, rows per wave, columns per lane, input group size, groups per load)
#define QTT_VALU_SHAPES(X)   \
  X(40, 8, 24, 1, 8, 1)      \
  X(41, 4, 24, 2, 8, 1)      \
  X(42, 4, 32, 1, 8, 1)      \
  X(43, 4, 16, 1, 8, 1)      \
  X(44, 8, 16, 1, 8, 1)      \
  X(45, 1, 8, 4, 8, 1)       \
  X(46, 2, 8, 2, 8, 1)       \
  X(47, 1, 8, 2, 8, 1)       \
  X(48, 4, 16, 1, 1, 1)      \
  X(49, 1, 8, 2, 8, 2)

void add_valu_kernels(std::vector<ValuCfg>& v) {
#define QTT_ADDV(id, nw, rw, cpl, nj, lg) \
  v.push_back({id, nw, rw, cpl, nj, lg, reinterpret_cast<const void*>(&core_step_valu64_kernel<nw, rw, cpl, nj, lg>), 0});
  QTT_VALU_SHAPES(QTT_ADDV)
#undef QTT_ADDV
}

// FP32 last core: one wave of 8 rows, 2 columns per lane, 128-byte loads
// (4 groups of 8 values)
ValuCfg valu32_last_cfg() {
  return {39, 1, 8, 2, 8, 4, reinterpret_cast<const void*>(&core_step_valu32_last_kernel<8, 2, 32>), 0};
}

const void* smallk_kernel(int dt) {
  switch (dt) {
    case 0: return reinterpret_cast<const void*>(&core_step_smallk_kernel<double>);
    case 1: return reinterpret_cast<const void*>(&core_step_smallk_kernel<float>);
    case 3: return reinterpret_cast<const void*>(&core_step_smallk_rows_kernel<bf16_tag, 8>);
    case 4: return reinterpret_cast<const void*>(&core_step_smallk_rows_kernel<float, 8>);
    default: return reinterpret_cast<const void*>(&core_step_smallk_kernel<bf16_tag>);
  }
}

}  // namespace qtt
