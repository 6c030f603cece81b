// Fused separable a-trous level (Section 3.3), binary16 storage.
#include "atrous_impl.h"

namespace sv {
bool launch_hv_f16(const HvArgs &a, bool unit, int rows, hipStream_t s) {
    return launch_hv<half_t>(a, unit, rows, s);
}
}  // namespace sv
