// Tile configurations of the generic, streamed and 4x4x4 core-step kernels,
// shared by the per-dtype kernel units.
#pragma once

#include <type_traits>
#include <vector>

#include "qtt_registry.hpp"

namespace qtt {


template <class Tc, class Tin, int WRW, int WCW, int WR, int WC, int KC, bool ROL, bool VEC, int KIND,
          int MINW = 1, int PF = 1, bool AHEAD = true>
inline KernelCfg make_cfg(int dt, bool in_f64, int id) {
  KernelCfg k;
  k.dt = dt;
  k.in_f64 = in_f64;
  k.vec = VEC;
  k.TR = 16 * WR * WRW;
  k.TC = (KIND >= 3 ? 4 : 16) * WC * WCW;
  k.KC = KC;
  k.NT = 64 * WRW * WCW;
  k.id = id;
  k.kind = KIND;
  if constexpr (KIND == 3) {
    static_assert(std::is_same<Tc, double>::value && std::is_same<Tin, double>::value,
                  "the 4x4x4 kernel is FP64 only");
    k.fn = reinterpret_cast<const void*>(&core_step_f64q_kernel<WRW, WCW, WR, WC, KC, PF, MINW, AHEAD>);
  } else if constexpr (KIND == 2)
    k.fn = reinterpret_cast<const void*>(&core_step_stream_kernel<Tc, Tin, WRW, WCW, WR, WC, KC, ROL, VEC, MINW>);
  else
    k.fn = reinterpret_cast<const void*>(&core_step_kernel<Tc, Tin, WRW, WCW, WR, WC, KC, ROL, VEC>);
  k.occ = 0;
  return k;
}

// Tile shapes: (id, waves along rows, waves along columns, row blocks per
// wave, column blocks per wave, rows on lanes).  Ids below 10 use the
// single-operand-LDS kernel, ids from 10 the pipelined two-operand kernel.
#define QTT_SHAPES_V1(X)     \
  X(0, 4, 1, 4, 4, true)     \
  X(1, 4, 1, 3, 4, true)     \
  X(2, 1, 4, 1, 4, false)    \
  X(5, 4, 1, 4, 2, true)     \
  X(6, 2, 2, 2, 2, true)
#define QTT_SHAPES_V3(X)     \
  X(20, 4, 1, 4, 4, true)    \
  X(21, 4, 1, 4, 2, true)    \
  X(22, 4, 1, 3, 4, true)    \
  X(23, 1, 4, 1, 4, false)   \
  X(24, 2, 2, 4, 4, true)    \
  X(25, 4, 1, 2, 4, true)    \
  X(26, 4, 1, 4, 1, true)    \
  X(27, 1, 4, 1, 2, false)
// FP64 shapes on the 4x4x4 instruction (ids from 60): (id, waves along rows,
// waves along columns, row blocks per wave, 4-column groups per wave, chunk
// length KC, core prefetch depth in steps, minimum resident waves per SIMD).
// They serve a core only when its step count is a multiple of KC / 4.
#define QTT_SHAPES_Q(X)             \
  X(60, 4, 1, 4, 8, 32, 2, 2)       \
  X(61, 4, 1, 4, 8, 32, 4, 2)       \
  X(62, 4, 1, 4, 8, 32, 8, 2)       \
  X(63, 4, 1, 3, 8, 32, 2, 2)       \
  X(64, 4, 1, 3, 8, 32, 4, 2)       \
  X(65, 4, 1, 4, 4, 32, 4, 2)       \
  X(66, 4, 1, 4, 4, 32, 8, 2)       \
  X(67, 4, 1, 3, 8, 8, 2, 2)        \
  X(68, 4, 1, 4, 8, 8, 2, 2)        \
  X(69, 2, 2, 4, 4, 32, 4, 2)
// the same without reading input fragments a step ahead (ids from 75)
#define QTT_SHAPES_QN(X)            \
  X(75, 4, 1, 4, 8, 32, 4, 2)       \
  X(76, 4, 1, 4, 8, 32, 8, 2)       \
  X(77, 4, 1, 3, 8, 32, 4, 2)       \
  X(78, 4, 1, 4, 6, 32, 4, 2)       \
  X(79, 4, 1, 4, 6, 32, 8, 2)

template <class Tc, class Tin, int KC1, int KC2>
inline void add_family(std::vector<KernelCfg>& v, int dt, bool in_f64) {
#define QTT_ADD1(id, a, b, c, d, rol) v.push_back(make_cfg<Tc, Tin, a, b, c, d, KC1, rol, true, 0>(dt, in_f64, id));
#define QTT_ADD3(id, a, b, c, d, rol) v.push_back(make_cfg<Tc, Tin, a, b, c, d, KC1, rol, true, 2>(dt, in_f64, id));
  QTT_SHAPES_V1(QTT_ADD1)
  QTT_SHAPES_V3(QTT_ADD3)
  // streamed shapes held to 3 resident waves per SIMD (fewer registers each)
  v.push_back(make_cfg<Tc, Tin, 4, 1, 4, 2, KC1, true, true, 2, 3>(dt, in_f64, 28));
  v.push_back(make_cfg<Tc, Tin, 4, 1, 2, 4, KC1, true, true, 2, 3>(dt, in_f64, 29));
  if constexpr (std::is_same<Tc, double>::value) {
#define QTT_ADDQ(id, a, b, c, d, kc, pf, mw) \
    v.push_back(make_cfg<Tc, Tin, a, b, c, d, kc, true, true, 3, mw, pf>(dt, in_f64, id));
    QTT_SHAPES_Q(QTT_ADDQ)
#undef QTT_ADDQ
#define QTT_ADDQN(id, a, b, c, d, kc, pf, mw) \
    v.push_back(make_cfg<Tc, Tin, a, b, c, d, kc, true, true, 3, mw, pf, false>(dt, in_f64, id));
    QTT_SHAPES_QN(QTT_ADDQN)
#undef QTT_ADDQN
  }
#undef QTT_ADD1
#undef QTT_ADD3
  // scalar-load fallback for shapes whose columns are not 16-byte aligned
  v.push_back(make_cfg<Tc, Tin, 2, 2, 2, 2, KC1, true, false, 0>(dt, in_f64, kGenericShape));
}


}  // namespace qtt
