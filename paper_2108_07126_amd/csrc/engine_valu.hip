// VALU engine dispatch (the kernels are instantiated per element type and
// dimension in the engine_valu_*.hip units so they compile in parallel).
#include "pm_internal.h"

namespace pm {

hipError_t launch_valu_f64_2(const PropParams& p, hipStream_t stream);
hipError_t launch_valu_f64_4(const PropParams& p, hipStream_t stream);
hipError_t launch_valu_f32_2(const PropParams& p, hipStream_t stream);
hipError_t launch_valu_f32_4(const PropParams& p, hipStream_t stream);

hipError_t launch_valu(int D, bool fp64, const PropParams& p, hipStream_t stream) {
    switch (D) {
        case 2: return fp64 ? launch_valu_f64_2(p, stream) : launch_valu_f32_2(p, stream);
        case 4: return fp64 ? launch_valu_f64_4(p, stream) : launch_valu_f32_4(p, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pm
