// A-trous pass kernels instantiated for one storage type and direction
// (separate compilation units so that they build in parallel).
#include "atrous_impl.h"

namespace sv {
void launch_pass_f32_2da(const AtrousArgs &a, bool unit, TileCfg cfg, hipStream_t s) {
    launch_pass<float, kDir2DA>(a, unit, cfg, s);
}
}  // namespace sv
