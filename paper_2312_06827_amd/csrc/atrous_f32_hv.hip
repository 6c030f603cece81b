// Fused separable a-trous level (Section 3.3), binary32 storage.
#include "atrous_impl.h"

namespace sv {
bool launch_hv_f32(const HvArgs &a, bool unit, int rows, hipStream_t s) {
    return launch_hv<float>(a, unit, rows, s);
}
}  // namespace sv
