// Composition of the denoised channels with the direct lighting (Section 3,
// step 7): out = direct * shadow + specular, per colour channel.
#include "sv_internal.h"

namespace sv {

struct ComposeArgs {
    const void *dr, *dg, *db, *sr, *sg, *sb, *pr, *pg, *pb;
    void *or_, *og, *ob;
    int w, h, pitch;
};

template <typename T, bool SHADOW, bool SPEC>
__global__ __launch_bounds__(256) void compose_k(ComposeArgs a) {
    const int x = (int)blockIdx.x * 64 + (int)(threadIdx.x & 63);
    const int y = (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6);
    if (x >= a.w || y >= a.h) return;
    const uint32_t o = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
    const void *d[3] = {a.dr, a.dg, a.db}, *sh[3] = {a.sr, a.sg, a.sb}, *sp[3] = {a.pr, a.pg, a.pb};
    void *out[3] = {a.or_, a.og, a.ob};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float v = ldo<T>(d[c], o);
        const float s = SHADOW ? ldo<T>(sh[c], o) : 1.f;
        const float p = SPEC ? ldo<T>(sp[c], o) : 0.f;
        sto<T>(out[c], o, fmaf(v, s, p));
    }
}

template <typename T>
static void launch(const ComposeArgs &a, bool shadow, bool spec, hipStream_t s) {
    dim3 grid((unsigned)((a.w + 63) / 64), (unsigned)((a.h + 3) / 4));
    if (shadow && spec) hipLaunchKernelGGL((compose_k<T, true, true>), grid, dim3(256), 0, s, a);
    else if (shadow) hipLaunchKernelGGL((compose_k<T, true, false>), grid, dim3(256), 0, s, a);
    else if (spec) hipLaunchKernelGGL((compose_k<T, false, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((compose_k<T, false, false>), grid, dim3(256), 0, s, a);
}

}  // namespace sv

extern "C" int sv_compose(const sv_rgb *direct, const sv_rgb *shadow, const sv_rgb *spec,
                          const sv_rgb *out, sv_dims d, sv_dtype t, sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    const int dc = check_dims(d);
    if (dc < 0 || !direct || !out) return SV_EINVAL;
    if (dc == 1) return SV_OK;
    const sv_rgb *ins[] = {direct, shadow, spec};
    for (const sv_rgb *p : ins)
        if (p && (!p->r || !p->g || !p->b)) return SV_EINVAL;
    if (!out->r || !out->g || !out->b) return SV_EINVAL;
    const size_t es = elem_size(t);
    const void *op[3] = {out->r, out->g, out->b};
    const span os[] = {plane_span(op[0], d, es), plane_span(op[1], d, es),
                       plane_span(op[2], d, es)};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (overlaps(os[i], os[j])) return SV_EALIAS;
    // an output plane may be the same plane as its own channel's input
    // (each pixel reads then writes its own element), but must not overlap
    // any other plane
    for (const sv_rgb *p : ins) {
        if (!p) continue;
        const void *pl[3] = {p->r, p->g, p->b};
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k) {
                const span si = plane_span(pl[c], d, es);
                if (overlaps(os[k], si) && !(k == c && pl[c] == op[k])) return SV_EALIAS;
            }
    }
    ComposeArgs a{direct->r, direct->g, direct->b,
                  shadow ? shadow->r : nullptr, shadow ? shadow->g : nullptr,
                  shadow ? shadow->b : nullptr, spec ? spec->r : nullptr,
                  spec ? spec->g : nullptr, spec ? spec->b : nullptr,
                  out->r, out->g, out->b, d.w, d.h, d.pitch};
    hipStream_t s = as_stream(stream);
    if (t == SV_F32) launch<float>(a, shadow != nullptr, spec != nullptr, s);
    else launch<half_t>(a, shadow != nullptr, spec != nullptr, s);
    return hip_status(hipGetLastError());
}
