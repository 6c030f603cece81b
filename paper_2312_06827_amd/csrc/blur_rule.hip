// Control bytes of the adaptive a-trous levels from per-pixel surface
// roughness and shadow angle: the coarser start of Section 3.2 and the
// roughness -> iteration count table of Section 3.5.
#include "sv_internal.h"

namespace sv {

struct RuleArgs {
    const float *rough, *angle;
    uint8_t *ctl;
    int w, h, pitch;
    sv_blur_rule r;
};

__global__ __launch_bounds__(256) void blur_rule_k(RuleArgs a) {
    const int x = (int)blockIdx.x * 64 + (int)(threadIdx.x & 63);
    const int y = (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6);
    if (x >= a.w || y >= a.h) return;
    const uint32_t o = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
    const float rg = a.rough ? ldf(a.rough, o) : 0.f;
    const float an = a.angle ? ldf(a.angle, o) : 0.f;
    bool shift = false;
    if (a.r.flags & SV_BR_SHIFT)
        shift = (a.rough && rg > a.r.rough_shift) || (a.angle && an > a.r.angle_shift);
    int levels = 15;
    if (a.r.flags & SV_BR_TABLE)
        levels = rg <= a.r.rough_none ? a.r.it_none : rg <= a.r.rough_one ? a.r.it_one : a.r.it_rest;
    a.ctl[o] = (uint8_t)((shift ? SV_CTL_SHIFT : 0) | levels);
}

}  // namespace sv

extern "C" int sv_blur_control(const float *roughness, const float *shadow_angle, uint8_t *ctl,
                               sv_dims d, const sv_blur_rule *r, sv_stream stream) {
    using namespace sv;
    const int dc = check_dims(d);
    if (dc < 0 || !r) return SV_EINVAL;
    const int its[] = {r->it_none, r->it_one, r->it_rest};
    for (int v : its)
        if (v < 0 || v > 15) return SV_EINVAL;
    if ((r->flags & ~(SV_BR_SHIFT | SV_BR_TABLE)) != 0) return SV_EINVAL;
    if ((r->flags & SV_BR_TABLE) && !roughness) return SV_EINVAL;
    if ((r->flags & SV_BR_SHIFT) && !roughness && !shadow_angle) return SV_EINVAL;
    if (dc == 1) return SV_OK;
    if (!ctl) return SV_EINVAL;
    const span out = plane_span(ctl, d, 1);
    if ((roughness && overlaps(out, plane_span(roughness, d, 4))) ||
        (shadow_angle && overlaps(out, plane_span(shadow_angle, d, 4))))
        return SV_EALIAS;
    RuleArgs a{roughness, shadow_angle, ctl, d.w, d.h, d.pitch, *r};
    dim3 grid((unsigned)((d.w + 63) / 64), (unsigned)((d.h + 3) / 4));
    hipLaunchKernelGGL(blur_rule_k, grid, dim3(256), 0, as_stream(stream), a);
    return hip_status(hipGetLastError());
}
