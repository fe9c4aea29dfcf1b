// VALU engine instantiation: float, dimension 4.
#include "valu_kernel.h"

namespace pm {
hipError_t launch_valu_f32_4(const PropParams& p, hipStream_t stream) {
    return launch_valu_one<float, 4>(p, stream);
}
}  // namespace pm
