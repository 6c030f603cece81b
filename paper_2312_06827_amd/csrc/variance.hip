// Variance estimate (Section 2): the temporal variance of the luminance
// moments where the history is long enough, a depth- and normal-weighted
// spatial estimate where it is not.
#include "sv_internal.h"

namespace sv {

struct VarianceArgs {
    const float *m1, *m2;
    const uint8_t *n;
    const void *z, *dzdx, *dzdy, *nx, *ny, *nz;
    float *var;
    int w, h, pitch;
    float sigma_z, sigma_n, eps_z, dmin;
    int min_hist, radius;
};

template <typename T>
__device__ __noinline__ float spatial_variance(const VarianceArgs &a, int x, int y, size_t o) {
    const float zp = ld((const T *)a.z + o), gx = ld((const T *)a.dzdx + o),
                gy = ld((const T *)a.dzdy + o);
    const float nxp = ld((const T *)a.nx + o), nyp = ld((const T *)a.ny + o),
                nzp = ld((const T *)a.nz + o);
    const int R = a.radius;
    // pass 1: weighted mean of m1
    float sw = 0.f, s1 = 0.f;
    for (int dy = -R; dy <= R; ++dy) {
        const int qy = y + dy;
        if (qy < 0 || qy >= a.h) continue;
        for (int dx = -R; dx <= R; ++dx) {
            const int qx = x + dx;
            if (qx < 0 || qx >= a.w) continue;
            const size_t q = (size_t)qy * a.pitch + qx;
            const float zq = ld((const T *)a.z + q);
            if (empty_px(zq)) continue;
            float wq = 1.f;
            if (dx != 0 || dy != 0) {
                const float den = fmaf(a.sigma_z, fabsf(fmaf(gx, (float)dx, gy * (float)dy)), a.eps_z);
                const float d = fmaf(nzp, ld((const T *)a.nz + q),
                                     fmaf(nyp, ld((const T *)a.ny + q), nxp * ld((const T *)a.nx + q)));
                const float e = -fabsf(zp - zq) / den * kLog2e +
                                a.sigma_n * fast_log2(fmaxf(d, a.dmin));
                wq = fast_exp2(e);
            }
            sw += wq;
            s1 = fmaf(wq, a.m1[q], s1);
        }
    }
    const float mean1 = s1 / sw;
    // pass 2: weighted within-pixel variance plus spread of m1
    float within = 0.f, spread = 0.f;
    for (int dy = -R; dy <= R; ++dy) {
        const int qy = y + dy;
        if (qy < 0 || qy >= a.h) continue;
        for (int dx = -R; dx <= R; ++dx) {
            const int qx = x + dx;
            if (qx < 0 || qx >= a.w) continue;
            const size_t q = (size_t)qy * a.pitch + qx;
            const float zq = ld((const T *)a.z + q);
            if (empty_px(zq)) continue;
            float wq = 1.f;
            if (dx != 0 || dy != 0) {
                const float den = fmaf(a.sigma_z, fabsf(fmaf(gx, (float)dx, gy * (float)dy)), a.eps_z);
                const float d = fmaf(nzp, ld((const T *)a.nz + q),
                                     fmaf(nyp, ld((const T *)a.ny + q), nxp * ld((const T *)a.nx + q)));
                const float e = -fabsf(zp - zq) / den * kLog2e +
                                a.sigma_n * fast_log2(fmaxf(d, a.dmin));
                wq = fast_exp2(e);
            }
            const float m1q = a.m1[q];
            within = fmaf(wq, fmaf(-m1q, m1q, a.m2[q]), within);
            const float dm = m1q - mean1;
            spread = fmaf(wq * dm, dm, spread);
        }
    }
    return fmaxf(0.f, (within + spread) / sw);
}

template <typename T>
__global__ __launch_bounds__(256) void variance_k(VarianceArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.w || y >= a.h) return;
    const size_t o = (size_t)y * a.pitch + x;
    const int n = a.n[o];
    float v = 0.f;
    if (n >= 1 && !empty_px(ld((const T *)a.z + o))) {
        if (n >= a.min_hist) {
            const float m1 = a.m1[o];
            v = fmaxf(0.f, fmaf(-m1, m1, a.m2[o]));
        } else {
            v = spatial_variance<T>(a, x, y, o);
        }
    }
    a.var[o] = v;
}

}  // namespace sv

extern "C" int sv_variance(const float *m1, const float *m2, const uint8_t *n, const sv_gbuf *g,
                           float *var, sv_dims d, sv_dtype t, const sv_variance_params *p,
                           sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    int dc = check_dims(d);
    if (dc < 0 || !g || !p) return SV_EINVAL;
    if (p->radius < 0 || p->radius > 7 || p->min_hist < 0) return SV_EINVAL;
    if (!(p->sigma_n >= 0.f)) return SV_EINVAL;
    if (dc == 1) return SV_OK;
    if (!m1 || !m2 || !n || !var || !g->z || !g->dzdx || !g->dzdy || !g->nx || !g->ny || !g->nz)
        return SV_EINVAL;
    const size_t es = elem_size(t);
    const span ins[] = {plane_span(m1, d, 4), plane_span(m2, d, 4), plane_span(n, d, 1),
                        plane_span(g->z, d, es), plane_span(g->dzdx, d, es),
                        plane_span(g->dzdy, d, es), plane_span(g->nx, d, es),
                        plane_span(g->ny, d, es), plane_span(g->nz, d, es)};
    const span so = plane_span(var, d, 4);
    for (const span &si : ins)
        if (overlaps(so, si)) return SV_EALIAS;
    // sigma_n == 0 turns the normal weight off: max(d, 1) makes log2 zero
    VarianceArgs a{m1, m2, n, g->z, g->dzdx, g->dzdy, g->nx, g->ny, g->nz, var,
                   d.w, d.h, d.pitch, p->sigma_z, p->sigma_n, p->eps_z,
                   p->sigma_n == 0.f ? 1.f : 0.f, p->min_hist, p->radius};
    dim3 grid((d.w + 63) / 64, (d.h + 3) / 4);
    if (t == SV_F32)
        hipLaunchKernelGGL(variance_k<float>, grid, dim3(256), 0, as_stream(stream), a);
    else
        hipLaunchKernelGGL(variance_k<half_t>, grid, dim3(256), 0, as_stream(stream), a);
    return hip_status(hipGetLastError());
}
