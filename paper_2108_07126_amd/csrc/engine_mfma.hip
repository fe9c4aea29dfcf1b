// MFMA engine: the non-paired instances of the propagation kernel and the
// dispatch over dimension, precision, method, pairing and integrator.
#include "mfma_kernel.h"

namespace pm {

template <typename T, int PMODE>
hipError_t launch_dims(int D, const PropParams& p, hipStream_t stream) {
    switch (D) {
        case 16: return launch_method<T, 16, kNT16, PMODE>(p, stream);
        case 32: return launch_method<T, 32, 1, PMODE>(p, stream);
        case 64: return launch_method<T, 64, 1, PMODE>(p, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mfma_pair(int precision, const PropParams& p, hipStream_t stream);
hipError_t launch_mfma_m6(int D, const PropParams& p, hipStream_t stream);

hipError_t launch_mfma(int D, int precision, const PropParams& p, hipStream_t stream) {
    if (p.order == kOrderM6) {
        if (precision != PM_FP64 || p.pair) return hipErrorInvalidValue;
        return launch_mfma_m6(D, p, stream);
    }
    if (p.pair) {
        if (D != 16) return hipErrorInvalidValue;
        return launch_mfma_pair(precision, p, stream);
    }
    switch (precision) {
        case PM_FP64: return launch_dims<double, 0>(D, p, stream);
        case PM_FP32: return launch_dims<float, 0>(D, p, stream);
        case PM_FP32_3M: return launch_dims<float, 1>(D, p, stream);
        case PM_BF16_SPLIT: return launch_dims<float, 2>(D, p, stream);
        default: return hipErrorInvalidValue;
    }
}

int mfma_chains_per_block(int D) { return D == 16 ? kNT16 : 1; }

}  // namespace pm
