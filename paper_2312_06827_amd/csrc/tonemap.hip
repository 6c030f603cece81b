// Reinhard tone map before denoising and its inverse after (Section 3.4).
#include "sv_internal.h"

namespace sv {

struct TonemapArgs {
    const void *r, *g, *b;
    void *ro, *go, *bo;
    int w, h, pitch;
    float k, weight;
    int mode, inverse;
};

template <typename T>
__global__ __launch_bounds__(256) void tonemap_k(TonemapArgs a) {
    int x = blockIdx.x * 64 + (threadIdx.x & 63);
    int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.w || y >= a.h) return;
    uint32_t o = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
    float r = ldo<T>(a.r, o), g = ldo<T>(a.g, o), b = ldo<T>(a.b, o);
    if (a.mode == SV_TM_CHANNEL) {
        if (!a.inverse) {
            r = r / (1.0f + a.k * r);
            g = g / (1.0f + a.k * g);
            b = b / (1.0f + a.k * b);
        } else {
            r = r / fmaxf(1.0f - a.k * r, 0x1p-20f);
            g = g / fmaxf(1.0f - a.k * g, 0x1p-20f);
            b = b / fmaxf(1.0f - a.k * b, 0x1p-20f);
        }
    } else if (!a.inverse) {
        float den = 1.0f + a.k * luma(r, g, b);
        r = r / den;
        g = g / den;
        b = b / den;
    } else if (a.mode == SV_TM_PAPER) {
        float s = (1.0f + luma(r, g, b)) * a.weight;
        r *= s;
        g *= s;
        b *= s;
    } else {
        inv_tonemap(r, g, b, a.k);
    }
    sto<T>(a.ro, o, r);
    sto<T>(a.go, o, g);
    sto<T>(a.bo, o, b);
}

}  // namespace sv

extern "C" int sv_tonemap(const sv_rgb *in, const sv_rgb *out, sv_dims d, sv_dtype t,
                          int inverse, const sv_tm_params *p, sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    int dc = check_dims(d);
    if (dc < 0 || !in || !out || !p) return SV_EINVAL;
    if (p->mode < SV_TM_LUMA || p->mode > SV_TM_PAPER) return SV_EINVAL;
    if (p->mode == SV_TM_PAPER && !inverse) return SV_EUNSUPPORTED;
    if (dc == 1) return SV_OK;
    if (!in->r || !in->g || !in->b || !out->r || !out->g || !out->b) return SV_EINVAL;
    TonemapArgs a{in->r, in->g, in->b, out->r, out->g, out->b, d.w, d.h, d.pitch,
                  p->k, p->weight, p->mode, inverse ? 1 : 0};
    dim3 grid((d.w + 63) / 64, (d.h + 3) / 4);
    if (t == SV_F32)
        hipLaunchKernelGGL(tonemap_k<float>, grid, dim3(256), 0, as_stream(stream), a);
    else
        hipLaunchKernelGGL(tonemap_k<half_t>, grid, dim3(256), 0, as_stream(stream), a);
    return hip_status(hipGetLastError());
}
