// MFMA engine: the slice-pair instances of the propagation kernel (one-wave
// 16-wide tiles carrying two slices of dimension <= 8, Taylor series).
#include "mfma_kernel.h"

namespace pm {

hipError_t launch_mfma_pair(int precision, const PropParams& p, hipStream_t stream) {
    switch (precision) {
        case PM_FP64: return launch_bl<double, 16, kNT16, 0, false, true>(p, stream);
        case PM_FP32: return launch_bl<float, 16, kNT16, 0, false, true>(p, stream);
        case PM_FP32_3M: return launch_bl<float, 16, kNT16, 1, false, true>(p, stream);
        case PM_BF16_SPLIT: return launch_bl<float, 16, kNT16, 2, false, true>(p, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pm
