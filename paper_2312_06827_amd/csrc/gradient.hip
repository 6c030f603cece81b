// Temporal gradient (A-SVGF), the answer to temporal lag that the paper's
// related work names (Section 2): one surface sample per 3x3 stratum of the
// previous frame is carried forward into the current frame and traced
// again there with its old random numbers; the change of its shading,
// reconstructed densely over 3x3 cells, raises the temporal blend factor
// where the lighting changed.
//
// Passes (one stream, graph-capturable: the key clear is a kernel):
//   grad_clear_k    cell keys := none
//   grad_project_k  per stratum: land the sample, atomicMin of its index
//                   on the cell's key (the lowest stratum index wins), and
//                   the sample's luminance difference and maximum, stored
//                   by stratum
//   grad_level_k    `levels` 5x5 B3 a-trous passes over the cells with a
//                   depth edge weight, on (delta, norm, present) alike, in
//                   LDS tiles (see below): the first gathers each cell's
//                   winning stratum (difference, maximum, presence), the
//                   last sets every pixel's blend factor from its cell,
//                   lambda = min(1, |delta| / norm) and
//                   alpha' = alpha + lambda (1 - alpha)
// With no level, or past step 32, the same steps run as per-cell passes
// (grad_gather_k, grad_atrous_k per level, grad_alpha_k per pixel).
//
// The normalized convolution is carried in a form with no underflow.  A
// cell holds (d, m, l): the weighted means of delta and norm over the
// samples that reached it and l = log2 of their total weight (-inf: none).
// A level combines its 25 taps in the log domain, each tap's exponent
// (kernel coefficient, depth weight, l of the tap) shifted by the largest,
// and yields the new means and l = that maximum + log2 of the shifted sum.
// In exact arithmetic this is the plain convolution of (delta p, norm p, p)
// with the means taken at the end; binary32 weights of a cell whose every
// neighbour lies far across depth edges (2^-150 and below) would underflow
// to zero there, and the cell would lose the ratio the plain sums define.
#include "sv_internal.h"

namespace sv {

namespace {

struct GradArgs {
    const void *pr, *pg, *pb, *rr, *rg, *rb;  // previous samples, traced again
    const void *fmvx, *fmvy, *fz;
    const uint8_t *pick;                      // cells: CH x CW, contiguous
    const void *z, *dzdx, *dzdy;              // current G-buffer
    float *alpha_map, *lambda;
    uint32_t *key;                            // cells: winning stratum
    float2 *samp;                             // strata: (lr - lp, max(lr, lp))
    float4 *ca, *cb;                          // cell ping-pong
    float4 *cz;                               // cells' centre pixel: z, dz/dx, dz/dy
    int w, h, pitch, cw, ch;
    float alpha, tau_z, sigma_z;
};

constexpr uint32_t kNone = 0xFFFFFFFFu;

__device__ __forceinline__ int cells_x(int w) { return (w + 2) / 3; }

__global__ __launch_bounds__(256) void grad_clear_k(uint32_t *key, int n) {
    const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (i < n) key[i] = kNone;
}

// The stratum's sample pixel q and where it lands; false if it does not.
template <typename T>
__device__ __forceinline__ bool land(const GradArgs &a, int s, int &qx, int &qy, int &cell) {
    const int sy = s / a.cw, sx = s - sy * a.cw;
    const int k = a.pick[s];
    qx = 3 * sx + k % 3;
    qy = 3 * sy + k / 3;
    if (k > 8 || qx >= a.w || qy >= a.h) return false;
    const uint32_t q = (uint32_t)qy * (uint32_t)a.pitch + (uint32_t)qx;
    // binary32 decisions with a fixed order, as the reprojection takes them
    const float tx = __fadd_rn(__fadd_rn((float)qx, ldo<T>(a.fmvx, q)), 0.5f);
    const float ty = __fadd_rn(__fadd_rn((float)qy, ldo<T>(a.fmvy, q)), 0.5f);
    if (!(tx >= 0.f && tx < (float)a.w && ty >= 0.f && ty < (float)a.h)) return false;
    const int px = (int)floorf(tx), py = (int)floorf(ty);
    const uint32_t p = (uint32_t)py * (uint32_t)a.pitch + (uint32_t)px;
    const float zc = ldo<T>(a.z, p);
    if (empty_px(zc)) return false;
    if (!(fabsf(__fsub_rn(ldo<T>(a.fz, q), zc)) <= __fmul_rn(a.tau_z, zc))) return false;
    cell = (py / 3) * a.cw + px / 3;
    return true;
}

template <typename T>
__global__ __launch_bounds__(256) void grad_project_k(GradArgs a) {
    const int s = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (s >= a.cw * a.ch) return;
    int qx, qy, cell;
    if (land<T>(a, s, qx, qy, cell)) {
        // the sample's luminances here, where its pixel is known: the
        // gather then reads one value per cell
        const uint32_t q = (uint32_t)qy * (uint32_t)a.pitch + (uint32_t)qx;
        const float lp = luma(ldo<T>(a.pr, q), ldo<T>(a.pg, q), ldo<T>(a.pb, q));
        const float lr = luma(ldo<T>(a.rr, q), ldo<T>(a.rg, q), ldo<T>(a.rb, q));
        a.samp[s] = make_float2(lr - lp, fmaxf(lr, lp));
        atomicMin(&a.key[cell], (uint32_t)s);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void grad_gather_k(GradArgs a) {
    const int c = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (c >= a.cw * a.ch) return;
    {  // the cell's centre pixel, which carries its depth in the reconstruction
        const int cy = c / a.cw, cx = c - cy * a.cw;
        const uint32_t o = (uint32_t)min(3 * cy + 1, a.h - 1) * (uint32_t)a.pitch +
                           (uint32_t)min(3 * cx + 1, a.w - 1);
        a.cz[c] = make_float4(ldo<T>(a.z, o), ldo<T>(a.dzdx, o), ldo<T>(a.dzdy, o), 0.f);
    }
    const uint32_t key = a.key[c];
    float4 v = make_float4(0.f, 0.f, -INFINITY, 0.f);  // (d, m, l): no sample
    if (key != kNone) {
        const float2 dm = a.samp[key];
        v = make_float4(dm.x, dm.y, 0.f, 0.f);  // one sample of weight 1
    }
    a.ca[c] = v;
}

// log2 of the B3-spline taps (1, 4, 6, 4, 1) / 16
__constant__ float kLog2B3[5] = {-4.0f, -2.0f, -1.4150374992788438f, -2.0f, -4.0f};

// One cascade level at cell step `step`: from `src` into `dst`, cells as
// (d, m, l) (see above).
__global__ __launch_bounds__(256) void grad_atrous_k(GradArgs a, const float4 *src, float4 *dst,
                                                    int step) {
    const int c = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (c >= a.cw * a.ch) return;
    const int cy = c / a.cw, cx = c - cy * a.cw;
    const float4 cc = a.cz[c];
    const float zc = cc.x, gx = cc.y, gy = cc.z;
    float e[25], d[25], m[25];
    float top = -INFINITY;
#pragma unroll
    for (int b = -2; b <= 2; ++b) {
#pragma unroll
        for (int k = -2; k <= 2; ++k) {
            const int t = (b + 2) * 5 + (k + 2);
            const int ny = cy + b * step, nx = cx + k * step;
            e[t] = -INFINITY;
            d[t] = m[t] = 0.f;
            if (ny < 0 || ny >= a.ch || nx < 0 || nx >= a.cw) continue;
            const int q = ny * a.cw + nx;
            const float4 v = src[q];
            if (!(v.z > -INFINITY)) continue;  // no sample reached that cell
            // offset between the centre pixels, in pixels
            const float ox = 3.f * (float)(k * step), oy = 3.f * (float)(b * step);
            const float den = fmaf(a.sigma_z, fabsf(grad_offset(gx, gy, ox, oy)), 1e-10f);
            e[t] = kLog2B3[b + 2] + kLog2B3[k + 2] - fabsf(zc - a.cz[q].x) * (kLog2e / den) + v.z;
            d[t] = v.x;
            m[t] = v.y;
            top = fmaxf(top, e[t]);
        }
    }
    float4 out = make_float4(0.f, 0.f, -INFINITY, 0.f);
    if (top > -INFINITY) {
        float sw = 0.f, sd = 0.f, sm = 0.f;
#pragma unroll
        for (int t = 0; t < 25; ++t) {
            const float w = exp2f(e[t] - top);  // 0 for a tap without samples
            sw += w;
            sd = fmaf(w, d[t], sd);
            sm = fmaf(w, m[t], sm);
        }
        out = make_float4(sd / sw, sm / sw, top + log2f(sw), 0.f);
    }
    dst[c] = out;
}

// ---- the cascade in LDS tiles ------------------------------------------------
//
// A level at cell step STEP as tiles of 64 consecutive cell columns by 4
// lattice rows of one phase (cell rows cy0 + j STEP), one cell per thread.
// The taps of those cells lie in the tile's own lattice rows (two above and
// below) and columns (2 STEP left and right), staged once in LDS: the cell
// (d, m, l) and the depth of its centre pixel.  The first level computes
// its cells from the projected samples while staging (the gather), the
// last writes the blend factor of each cell's 3 x 3 pixels (and lambda).
// Every tap is the same arithmetic as grad_atrous_k's, with the hardware
// exp2, log2 and reciprocal (each within an ulp; the weights are relative to
// the largest, whose exp2 is exactly 1).
constexpr int kGTX = 64, kGTY = 4;

// The cell (d, m, l) of cell c from its winning sample: one sample of
// weight 1 (l = 0), or none (l = -inf).
template <typename T>
__device__ __forceinline__ float4 cell_sample(const GradArgs &a, int c) {
    const uint32_t key = a.key[c];
    // no branch before the load (a cell without a sample reads stratum 0
    // and drops it), so that a thread's cells all have their loads in flight
    const bool none = key == kNone;
    const float2 dm = a.samp[none ? 0u : key];
    return none ? make_float4(0.f, 0.f, -INFINITY, 0.f) : make_float4(dm.x, dm.y, 0.f, 0.f);
}

// Offset of the centre pixel of cell (cx, cy).
__device__ __forceinline__ uint32_t cell_centre(const GradArgs &a, int cx, int cy) {
    return (uint32_t)min(3 * cy + 1, a.h - 1) * (uint32_t)a.pitch + (uint32_t)min(3 * cx + 1, a.w - 1);
}

template <typename T, int STEP>
__global__ __launch_bounds__(256) void grad_level_k(GradArgs a, const float4 *src, float4 *dst,
                                                    int first, int last) {
    constexpr int HX = 2 * STEP, COLS = kGTX + 2 * HX, ROWS = kGTY + 4, NS = ROWS * COLS;
    __shared__ float4 s_c[NS];  // (d, m, l)
    __shared__ float s_z[NS];   // depth of the cell's centre pixel
    const int gxt = (a.cw + kGTX - 1) / kGTX;
    const int t = xcd_tile(gxt * STEP * ((a.ch + STEP * kGTY - 1) / (STEP * kGTY)));
    if (t < 0) return;
    const int tyt = t / gxt, band = tyt / STEP, phase = tyt - band * STEP;
    const int cx0 = (t - tyt * gxt) * kGTX, cy0 = band * STEP * kGTY + phase;
    // staging: every load of a thread's cells issued before the first store
    constexpr int IT = (NS + 255) / 256;
    float4 v[IT];
    float zq[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = (int)threadIdx.x + it * 256;
        const int r = i / COLS, col = i - r * COLS;
        const int cx = cx0 - HX + col, cy = cy0 + (r - 2) * STEP;
        const bool in = i < NS && cx >= 0 && cx < a.cw && cy >= 0 && cy < a.ch;
        const int c = in ? cy * a.cw + cx : 0;
        v[it] = first ? cell_sample<T>(a, c) : src[c];
        zq[it] = ldo<T>(a.z, cell_centre(a, in ? cx : 0, in ? cy : 0));
        if (!in) {
            v[it] = make_float4(0.f, 0.f, -INFINITY, 0.f);
            zq[it] = 0.f;
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = (int)threadIdx.x + it * 256;
        if (i < NS) {
            s_c[i] = v[it];
            s_z[i] = zq[it];
        }
    }
    __syncthreads();
    const int lx = (int)(threadIdx.x & 63), ly = (int)(threadIdx.x >> 6);
    const int cx = cx0 + lx, cy = cy0 + ly * STEP;
    if (cx >= a.cw || cy >= a.ch) return;
    const int ci = (ly + 2) * COLS + HX + lx;
    const uint32_t o = cell_centre(a, cx, cy);
    const float zc = s_z[ci], gx = ldo<T>(a.dzdx, o), gy = ldo<T>(a.dzdy, o);
    float e[25];
    float top = -INFINITY;
#pragma unroll
    for (int b = -2; b <= 2; ++b)
#pragma unroll
        for (int k = -2; k <= 2; ++k) {
            const int q = ci + b * COLS + k * STEP;
            const float ox = 3.f * (float)(k * STEP), oy = 3.f * (float)(b * STEP);
            const float den = fmaf(a.sigma_z, fabsf(grad_offset(gx, gy, ox, oy)), 1e-10f);
            const float et = kLog2B3[b + 2] + kLog2B3[k + 2] -
                             fabsf(zc - s_z[q]) * (kLog2e * fast_rcp(den)) + s_c[q].z;
            e[(b + 2) * 5 + k + 2] = et;
            top = fmaxf(top, et);
        }
    float4 out = make_float4(0.f, 0.f, -INFINITY, 0.f);
    if (top > -INFINITY) {
        float sw = 0.f, sd = 0.f, sm = 0.f;
#pragma unroll
        for (int b = -2; b <= 2; ++b)
#pragma unroll
            for (int k = -2; k <= 2; ++k) {
                const float4 v = s_c[ci + b * COLS + k * STEP];
                const float w = fast_exp2(e[(b + 2) * 5 + k + 2] - top);  // 0 without samples
                sw += w;
                sd = fmaf(w, v.x, sd);
                sm = fmaf(w, v.y, sm);
            }
        const float inv = fast_rcp(sw);
        out = make_float4(quot(sd, sw, inv), quot(sm, sw, inv), top + fast_log2(sw), 0.f);
    }
    const int c = cy * a.cw + cx;
    if (!last) {
        dst[c] = out;
        return;
    }
    // the blend factor of the cell's pixels
    const float lam = (out.z > -INFINITY && out.y > 0.f) ? fminf(1.f, fabsf(out.x) / out.y) : 0.f;
    const float am = fmaf(lam, 1.f - a.alpha, a.alpha);
    for (int dy = 0; dy < 3; ++dy) {
        const int y = 3 * cy + dy;
        if (y >= a.h) break;
        for (int dx = 0; dx < 3; ++dx) {
            const int x = 3 * cx + dx;
            if (x < a.w) stf(a.alpha_map, (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x, am);
        }
    }
    if (a.lambda) a.lambda[c] = lam;
}

template <typename T>
bool launch_level(const GradArgs &a, const float4 *src, float4 *dst, int step, bool first,
                  bool last, hipStream_t s) {
    const int gxt = (a.cw + kGTX - 1) / kGTX;
    const int tiles = gxt * step * ((a.ch + step * kGTY - 1) / (step * kGTY));
    const dim3 g(xcd_grid(tiles)), b(256);
    const int f = first ? 1 : 0, l = last ? 1 : 0;
    switch (step) {
    case 1: hipLaunchKernelGGL((grad_level_k<T, 1>), g, b, 0, s, a, src, dst, f, l); return true;
    case 2: hipLaunchKernelGGL((grad_level_k<T, 2>), g, b, 0, s, a, src, dst, f, l); return true;
    case 4: hipLaunchKernelGGL((grad_level_k<T, 4>), g, b, 0, s, a, src, dst, f, l); return true;
    case 8: hipLaunchKernelGGL((grad_level_k<T, 8>), g, b, 0, s, a, src, dst, f, l); return true;
    case 16: hipLaunchKernelGGL((grad_level_k<T, 16>), g, b, 0, s, a, src, dst, f, l); return true;
    case 32: hipLaunchKernelGGL((grad_level_k<T, 32>), g, b, 0, s, a, src, dst, f, l); return true;
    default: return false;
    }
}

__global__ __launch_bounds__(256) void grad_alpha_k(GradArgs a, const float4 *cells) {
    const int x = (int)blockIdx.x * 64 + (int)(threadIdx.x & 63);
    const int y = (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6);
    if (x >= a.w || y >= a.h) return;
    const int c = (y / 3) * a.cw + x / 3;
    const float4 v = cells[c];  // (d, m, l): weighted means of delta and norm
    const float lam = (v.z > -INFINITY && v.y > 0.f) ? fminf(1.f, fabsf(v.x) / v.y) : 0.f;
    stf(a.alpha_map, (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x, fmaf(lam, 1.f - a.alpha, a.alpha));
    if (a.lambda && x % 3 == 0 && y % 3 == 0) a.lambda[c] = lam;
}

struct GradWork {
    size_t key, samp, ca, cb, cz, total;
};

GradWork work_layout(sv_dims d) {
    const size_t n = (size_t)((d.w + 2) / 3) * (size_t)((d.h + 2) / 3);
    const auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t f4 = up(n * sizeof(float4));
    GradWork g;
    g.key = 0;
    g.samp = up(n * sizeof(uint32_t));
    g.ca = g.samp + up(n * sizeof(float2));
    g.cb = g.ca + f4;
    g.cz = g.cb + f4;
    g.total = g.cz + n * sizeof(float4);
    return g;
}

// Levels at cell steps up to 32 run as LDS tiles, the first gathering the
// samples itself and the last writing the blend factors; with no level, or
// past step 32, the per-cell passes do those steps.
template <typename T>
void launch_gradient(GradArgs a, int levels, hipStream_t s) {
    const int n = a.cw * a.ch;
    const dim3 g1((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(grad_clear_k, g1, dim3(256), 0, s, a.key, n);
    hipLaunchKernelGGL(grad_project_k<T>, g1, dim3(256), 0, s, a);
    const bool tiled = levels >= 1 && levels <= 6;
    if (!tiled) hipLaunchKernelGGL(grad_gather_k<T>, g1, dim3(256), 0, s, a);
    float4 *src = a.ca, *dst = a.cb;
    for (int l = 0; l < levels; ++l) {
        if (tiled)
            launch_level<T>(a, src, dst, 1 << l, l == 0, l == levels - 1, s);
        else
            hipLaunchKernelGGL(grad_atrous_k, g1, dim3(256), 0, s, a, (const float4 *)src, dst,
                               1 << l);
        float4 *tmp = src;
        src = dst;
        dst = tmp;
    }
    if (!tiled)
        hipLaunchKernelGGL(grad_alpha_k,
                           dim3((unsigned)((a.w + 63) / 64), (unsigned)((a.h + 3) / 4)),
                           dim3(256), 0, s, a, (const float4 *)src);
}

}  // namespace

}  // namespace sv

extern "C" size_t sv_grad_work_bytes(sv_dims d) {
    if (sv::check_dims(d) < 0) return 0;
    return sv::work_layout(d).total;
}

extern "C" int sv_temporal_gradient(const sv_rgb *prev, const sv_rgb *reshade, const void *fmvx,
                                    const void *fmvy, const void *fz, const uint8_t *pick,
                                    const sv_gbuf *g, float *alpha_map, float *lambda, void *work,
                                    sv_dims d, sv_dtype t, const sv_grad_params *p,
                                    sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    const int dc = check_dims(d);
    if (dc < 0 || !prev || !reshade || !g || !p) return SV_EINVAL;
    if (p->levels < 0 || p->levels > 8 || !(p->tau_z >= 0.f) || !(p->sigma_z >= 0.f))
        return SV_EINVAL;
    if (dc == 1) return SV_OK;
    const void *req[] = {prev->r, prev->g, prev->b, reshade->r, reshade->g, reshade->b, fmvx,
                         fmvy, fz, pick, g->z, g->dzdx, g->dzdy, alpha_map, work};
    for (const void *q : req)
        if (!q) return SV_EINVAL;
    if ((uintptr_t)work % 16) return SV_EINVAL;  // float4 cells
    const int cw = (d.w + 2) / 3, ch = (d.h + 2) / 3;
    const size_t es = elem_size(t);
    const GradWork wl = work_layout(d);
    const span outs[] = {plane_span(alpha_map, d, 4),
                         span{(uintptr_t)work, (uintptr_t)work + wl.total},
                         lambda ? span{(uintptr_t)lambda, (uintptr_t)(lambda + (size_t)cw * ch)}
                                : span{0, 0}};
    const span ins[] = {plane_span(prev->r, d, es),    plane_span(prev->g, d, es),
                        plane_span(prev->b, d, es),    plane_span(reshade->r, d, es),
                        plane_span(reshade->g, d, es), plane_span(reshade->b, d, es),
                        plane_span(fmvx, d, es),       plane_span(fmvy, d, es),
                        plane_span(fz, d, es),         plane_span(g->z, d, es),
                        plane_span(g->dzdx, d, es),    plane_span(g->dzdy, d, es),
                        span{(uintptr_t)pick, (uintptr_t)(pick + (size_t)cw * ch)}};
    for (int i = 0; i < 3; ++i) {
        for (const span &si : ins)
            if (overlaps(outs[i], si)) return SV_EALIAS;
        for (int j = i + 1; j < 3; ++j)
            if (overlaps(outs[i], outs[j])) return SV_EALIAS;
    }
    unsigned char *wb = (unsigned char *)work;
    GradArgs a{prev->r,    prev->g,    prev->b,   reshade->r,
               reshade->g, reshade->b, fmvx,      fmvy,
               fz,         pick,       g->z,      g->dzdx,
               g->dzdy,    alpha_map,  lambda,    (uint32_t *)(wb + wl.key),
               (float2 *)(wb + wl.samp), (float4 *)(wb + wl.ca), (float4 *)(wb + wl.cb),
               (float4 *)(wb + wl.cz), d.w, d.h, d.pitch, cw, ch, p->alpha, p->tau_z, p->sigma_z};
    hipStream_t s = as_stream(stream);
    if (t == SV_F32) launch_gradient<float>(a, p->levels, s);
    else launch_gradient<half_t>(a, p->levels, s);
    return hip_status(hipGetLastError());
}
