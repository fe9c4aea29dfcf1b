// VALU engine instantiation: double, dimension 2.
#include "valu_kernel.h"

namespace pm {
hipError_t launch_valu_f64_2(const PropParams& p, hipStream_t stream) {
    return launch_valu_one<double, 2>(p, stream);
}
}  // namespace pm
