// Group-product kernels for the 5-smooth transform sizes that are not powers of two (the
// half forms only: rows and columns that fill at most half of their transform, which the
// paper's layout of stations over prism centres always gives).  Instantiated per precision
// in group_mixed_f32.hip and group_mixed_f64.hip.
#pragma once
#include "group_kernels.h"

// 5-smooth multiples of 8 up to 640 that are not powers of two: the transform sizes of grids up
// to 320 x 320 stations over as many prism columns.
#define BTTB_MIXED_SIZES(X)                                                                          \
  X(24) X(40) X(48) X(72) X(80) X(96) X(120) X(144) X(160) X(192) X(200) X(216) X(240) X(288) X(320) \
  X(360) X(384) X(400) X(432) X(480) X(576) X(600) X(640)

namespace bttb {

template <typename T>
StageKernel<T> stage_kernel_mixed(int N, int st, bool fused, bool half) {
  if (!half) return nullptr;
  switch (N) {
#define BTTB_X(NN) \
  case NN: return stage_kernel_h<T, NN, true>(st, fused);
    BTTB_MIXED_SIZES(BTTB_X)
#undef BTTB_X
    default: return nullptr;
  }
}

}  // namespace bttb
