// FP64 group-product kernels of the 5-smooth sizes (group_mixed.h).
#include "group_mixed.h"

namespace bttb {

template StageKernel<double> stage_kernel_mixed<double>(int, int, bool, bool);

}  // namespace bttb
