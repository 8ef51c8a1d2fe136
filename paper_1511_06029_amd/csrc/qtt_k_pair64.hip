// Fused core pairs in FP64: one instantiation per boundary rank (24, 32,
// or padded 17..32), rows of the second core (<= 192 or 256) and first-core flag.
#define QTT_KERNEL_TEMPLATES_ONLY
#include "qtt_registry.hpp"

namespace qtt {

namespace {
// RA = 24 and 32 exact; "RA = 33" stands for the padded 256-row kernel.
template <int RA, int WRB, bool FIRST>
const void* fn() {
  constexpr int R = RA > 32 ? 32 : RA;
  return reinterpret_cast<const void*>(&core_pair_f64_kernel<R, WRB, FIRST, FIRST ? 8 : 32, 4, (RA > 32)>);
}
}  // namespace

const void* pair_f64_kernel(int f) {
  static const void* fns[12] = {fn<24, 3, false>(), fn<24, 4, false>(), fn<32, 3, false>(), fn<32, 4, false>(),
                                fn<33, 3, false>(), fn<33, 4, false>(), fn<24, 3, true>(),  fn<24, 4, true>(),
                                fn<32, 3, true>(),  fn<32, 4, true>(),  fn<33, 3, true>(),  fn<33, 4, true>()};
  return (f >= 0 && f < 12) ? fns[f] : nullptr;
}

}  // namespace qtt
