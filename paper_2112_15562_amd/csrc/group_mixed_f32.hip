// FP32 group-product kernels of the 5-smooth sizes (group_mixed.h).
#include "group_mixed.h"

namespace bttb {

bool mixed_size(int N) {
  switch (N) {
#define BTTB_X(NN) case NN:
    BTTB_MIXED_SIZES(BTTB_X)
#undef BTTB_X
    return true;
    default: return false;
  }
}

template StageKernel<float> stage_kernel_mixed<float>(int, int, bool, bool);

}  // namespace bttb
