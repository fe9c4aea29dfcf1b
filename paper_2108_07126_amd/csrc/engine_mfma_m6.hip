// MFMA engine: the sixth-order Magnus instances of the propagation kernel
// (FP64; Taylor or Chebyshev exponential).
#include "mfma_kernel.h"

namespace pm {

namespace {
template <int D, int NT>
hipError_t launch_m6(const PropParams& p, hipStream_t stream) {
    if (p.method == PM_EXPM_CHEBYSHEV) return launch_bl<double, D, NT, 0, true, false, true>(p, stream);
    return launch_bl<double, D, NT, 0, false, false, true>(p, stream);
}
}  // namespace

hipError_t launch_mfma_m6(int D, const PropParams& p, hipStream_t stream) {
    switch (D) {
        case 16: return launch_m6<16, kNT16>(p, stream);
        case 32: return launch_m6<32, 1>(p, stream);
        case 64: return launch_m6<64, 1>(p, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pm
