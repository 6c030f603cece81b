// Temporal filter: backward reprojection of the history, variance colour
// clamp of the reprojected colour, and accumulation of colour and luminance
// moments (Section 2; Section 3 step 4; Section 3.1).  One fused pass:
// every pixel reads its current colour (tone mapped on the fly), its 3x3
// neighbourhood through an LDS tile, and four bilinear history taps.
#include "sv_internal.h"

namespace sv {

constexpr int kTX = 64, kTY = 4;  // pixels per workgroup (one wave per row)

struct TemporalArgs {
    const void *cr, *cg, *cb;
    const void *z, *nx, *ny, *nz;
    const uint8_t *id;
    const void *mvx, *mvy;
    const void *pz, *pnx, *pny, *pnz;
    const uint8_t *pid;
    const void *hr, *hg, *hb;
    const float *hm1, *hm2c;  // E[L], E[L^2] - E[L]^2
    const uint8_t *hn;
    void *or_, *og, *ob;
    float *om1, *om2c;
    uint8_t *on;
    const float *alpha_map;
    int w, h, pitch;
    float alpha, alpha_m, gamma, tau_z, tau_n, tm_k;
    int max_hist;
    // feature mode only
    const void *dzdx, *dzdy, *alr, *alg, *alb;
    uint4 *feat;              // two 16-byte halves per pixel, row y * w + x
    float *fhr, *fhg, *fhb;   // clamped reprojected history (optional)
    const float *mu, *inv_s;  // standardisation
};

// binary32 decisions, operation order fixed and never contracted.
__device__ __forceinline__ bool depth_consistent(float z_prev, float z_cur, float tau) {
    float d = fabsf(__fsub_rn(z_prev, z_cur));
    float lim = __fmul_rn(tau, z_cur);
    return d <= lim;
}

__device__ __forceinline__ bool normal_consistent(float ax, float ay, float az, float bx, float by,
                                                  float bz, float tau) {
    float d = __fmul_rn(ax, bx);
    d = fmaf(ay, by, d);
    d = fmaf(az, bz, d);
    return d >= tau;
}

// 3x3 box of the tile around (lx+1, ly+1): clamp bounds mu -+ gamma sigma
// per channel from the mean and population variance over valid entries
// (w component 1, else 0; their colour is masked out here).  Binary64: the
// bounds are differences of quantities of the colour's size and may be
// close to zero.  One pass of sums of x and x^2 suffices there: products of
// binary32 values are exact in binary64, and the cancellation in
// E[x^2] - E[x]^2 costs at most log2(mu^2 / sigma^2) of its 53 bits.
__device__ __forceinline__ void box_bounds(const float4 *tile, int lx, int ly, float gamma,
                                           float3 &lo, float3 &hi) {
    double s1r = 0.0, s1g = 0.0, s1b = 0.0, s2r = 0.0, s2g = 0.0, s2b = 0.0;
    float cnt = 0.f;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const float4 q = tile[(ly + dy) * (kTX + 2) + lx + dx];
            const double r = q.w * q.x, g = q.w * q.y, b = q.w * q.z;  // exact: w is 0 or 1
            s1r += r;
            s1g += g;
            s1b += b;
            s2r = fma(r, r, s2r);
            s2g = fma(g, g, s2g);
            s2b = fma(b, b, s2b);
            cnt += q.w;
        }
    const double inv = 1.0 / (double)cnt;
    const double mr = s1r * inv, mg = s1g * inv, mb = s1b * inv;
    const double vr = fmax(0.0, fma(-mr, mr, s2r * inv));
    const double vg = fmax(0.0, fma(-mg, mg, s2g * inv));
    const double vb = fmax(0.0, fma(-mb, mb, s2b * inv));
    const double gr = gamma * sqrt(vr), gg = gamma * sqrt(vg), gb = gamma * sqrt(vb);
    lo = make_float3((float)(mr - gr), (float)(mg - gg), (float)(mb - gb));
    hi = make_float3((float)(mr + gr), (float)(mg + gg), (float)(mb + gb));
}

// Stage the current colour (tone mapped if TM) of the tile and a one-pixel
// apron; w = 1 for pixels inside the image that are not empty, else 0.
template <typename T, bool TM>
__device__ __forceinline__ void stage_current(float4 *tile, const void *cr, const void *cg,
                                              const void *cb, const void *zp, int w, int h,
                                              int pitch, float tm_k, int bx, int by) {
    // unrolled, every load issued from an in-image address (masked after)
    const int x0 = (int)bx * kTX - 1, y0 = (int)by * kTY - 1;
    constexpr int NS = (kTX + 2) * (kTY + 2), IT = (NS + 255) / 256;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = threadIdx.x + it * 256;
        const int r = i / (kTX + 2), c = i - r * (kTX + 2);
        const int gx = x0 + c, gy = y0 + r;
        const bool in = i < NS && gx >= 0 && gx < w && gy >= 0 && gy < h;
        const uint32_t o = in ? (uint32_t)gy * (uint32_t)pitch + (uint32_t)gx : 0u;
        float R = ldo<T>(cr, o), G = ldo<T>(cg, o), B = ldo<T>(cb, o);
        const float zz = zp ? ldo<T>(zp, o) : 1.f;
        if (TM) {
            const float sc = 1.0f / (1.0f + tm_k * luma(R, G, B));
            R *= sc;
            G *= sc;
            B *= sc;
        }
        if (i < NS)
            tile[i] = in ? make_float4(R, G, B, empty_px(zz) ? 0.f : 1.f)
                         : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Population variance of the luminance over the valid entries of the 3x3
// box around (lx+1, ly+1) (two passes, binary32).
__device__ __forceinline__ float box_luma_var(const float4 *tile, int lx, int ly) {
    float s = 0.f, cnt = 0.f, L[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float4 q = tile[(ly + i / 3) * (kTX + 2) + lx + i % 3];
        L[i] = luma(q.x, q.y, q.z);
        s = q.w > 0.f ? s + L[i] : s;
        cnt += q.w;
    }
    const float m = s / cnt;
    float v = 0.f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float4 q = tile[(ly + i / 3) * (kTX + 2) + lx + i % 3];
        const float d = L[i] - m;
        v = q.w > 0.f ? fmaf(d, d, v) : v;
    }
    return v / cnt;
}

__device__ __forceinline__ uint32_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return u >> 16;
}

// Standardise the 14 raw features, round to bfloat16 and store the pixel's
// 32-byte row (two zero pads at the end).
__device__ __forceinline__ void store_features(const TemporalArgs &a, int x, int y,
                                               const float (&f)[SV_MLP_IN]) {
    uint32_t pk[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k0 = 2 * i, k1 = 2 * i + 1;
        // features 14 and 15 are the zero pads
        const uint32_t lo = k0 < SV_MLP_IN ? bf16_bits((f[k0] - a.mu[k0]) * a.inv_s[k0]) : 0u;
        const uint32_t hi = k1 < SV_MLP_IN ? bf16_bits((f[k1] - a.mu[k1]) * a.inv_s[k1]) : 0u;
        pk[i] = lo | (hi << 16);
    }
    uint4 *row = a.feat + 2 * ((size_t)y * (size_t)a.w + (size_t)x);
    row[0] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
    row[1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
}

// One 64x4 tile (bx, by).  Returns once this thread's pixel is done (the
// caller's barrier follows).
template <typename T, bool TM, bool CLAMP, bool USE_ID, bool FEAT>
__device__ __forceinline__ void temporal_tile(const TemporalArgs &a, float4 *tile, int bx,
                                              int by) {
    stage_current<T, TM>(tile, a.cr, a.cg, a.cb, a.z, a.w, a.h, a.pitch, a.tm_k, bx, by);
    __syncthreads();
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int x = bx * kTX + lx, y = by * kTY + ly;
    if (x >= a.w || y >= a.h) return;
    const uint32_t o = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
    const float4 c = tile[(ly + 1) * (kTX + 2) + lx + 1];
    const float L = luma(c.x, c.y, c.z);
    const float zc = ldo<T>(a.z, o);
    if (FEAT && empty_px(zc)) {
        float f[SV_MLP_IN];
#pragma unroll
        for (int i = 0; i < SV_MLP_IN; ++i) f[i] = 0.f;
        store_features(a, x, y, f);
        if (a.fhr) {
            stf(a.fhr, o, 0.f);
            stf(a.fhg, o, 0.f);
            stf(a.fhb, o, 0.f);
        }
        return;
    }
    if (empty_px(zc)) {
        sto<T>(a.or_, o, c.x);
        sto<T>(a.og, o, c.y);
        sto<T>(a.ob, o, c.z);
        stf(a.om1, o, 0.f);
        stf(a.om2c, o, 0.f);
        a.on[o] = 0;
        return;
    }
    const float nxc = ldo<T>(a.nx, o), nyc = ldo<T>(a.ny, o),
                nzc = ldo<T>(a.nz, o);
    const float mvx = ldo<T>(a.mvx, o), mvy = ldo<T>(a.mvy, o);
    const uint8_t idc = USE_ID ? a.id[o] : 0;

    // ---- backward reprojection: bilinear taps around p + mv ----
    // Every load of the four taps is issued before any test, so the taps'
    // memory latencies overlap instead of chaining through the tests.
    float bw[4], tz[4], tnx[4], tny[4], tnz[4], tr[4], tg[4], tb[4], t1[4], t2[4];
    int thn[4], tid_[4];
    bool inb[4];
    const bool mv_ok = fabsf(mvx) < 1048576.0f && fabsf(mvy) < 1048576.0f;
    const float fx0 = mv_ok ? floorf(mvx) : 0.f, fy0 = mv_ok ? floorf(mvy) : 0.f;
    const float fx = mvx - fx0, fy = mvy - fy0;  // exact in binary32
    const int x0 = x + (int)fx0, y0 = y + (int)fy0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int tx = x0 + (t & 1), ty = y0 + (t >> 1);
        bw[t] = ((t & 1) ? fx : 1.0f - fx) * ((t >> 1) ? fy : 1.0f - fy);
        inb[t] = mv_ok && bw[t] > 0.f && tx >= 0 && tx < a.w && ty >= 0 && ty < a.h;
        const uint32_t q = inb[t] ? (uint32_t)ty * (uint32_t)a.pitch + (uint32_t)tx : o;
        thn[t] = a.hn[q];
        tz[t] = ldo<T>(a.pz, q);
        tnx[t] = ldo<T>(a.pnx, q);
        tny[t] = ldo<T>(a.pny, q);
        tnz[t] = ldo<T>(a.pnz, q);
        tid_[t] = USE_ID ? a.pid[q] : 0;
        tr[t] = ldo<T>(a.hr, q);
        tg[t] = ldo<T>(a.hg, q);
        tb[t] = ldo<T>(a.hb, q);
        t1[t] = ldf(a.hm1, q);
        t2[t] = ldf(a.hm2c, q);
    }
    float sw = 0.f, ar = 0.f, ag = 0.f, ab = 0.f, a1 = 0.f;
    int nmax = 0;
    bool ok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        ok[t] = inb[t] && thn[t] >= 1 && depth_consistent(tz[t], zc, a.tau_z) &&
                normal_consistent(tnx[t], tny[t], tnz[t], nxc, nyc, nzc, a.tau_n) &&
                (!USE_ID || tid_[t] == idc);
        // selects, not zero weights: an unusable tap's history may hold
        // anything (even NaN) and must not reach the sums
        sw = ok[t] ? sw + bw[t] : sw;
        ar = ok[t] ? fmaf(bw[t], tr[t], ar) : ar;
        ag = ok[t] ? fmaf(bw[t], tg[t], ag) : ag;
        ab = ok[t] ? fmaf(bw[t], tb[t], ab) : ab;
        a1 = ok[t] ? fmaf(bw[t], t1[t], a1) : a1;
        nmax = ok[t] ? max(nmax, thn[t]) : nmax;
    }
    const bool any = ok[0] || ok[1] || ok[2] || ok[3];
    float outr, outg, outb, m1, m2c;
    int n;
    if (FEAT && !any) {
        float f[SV_MLP_IN] = {L, 0.f, 0.f, box_luma_var(tile, lx, ly), 1.0f / 255.0f,
                              ldo<T>(a.dzdx, o), ldo<T>(a.dzdy, o), nxc, nyc, nzc,
                              mv_ok ? sqrtf(fmaf(mvy, mvy, mvx * mvx)) : 0.f,
                              ldo<T>(a.alr, o), ldo<T>(a.alg, o), ldo<T>(a.alb, o)};
        store_features(a, x, y, f);
        if (a.fhr) {
            stf(a.fhr, o, 0.f);
            stf(a.fhg, o, 0.f);
            stf(a.fhb, o, 0.f);
        }
        return;
    }
    if (!any) {
        outr = c.x;
        outg = c.y;
        outb = c.z;
        m1 = L;
        m2c = 0.f;
        n = 1;
    } else {
        const float inv = 1.0f / sw;
        float hr = ar * inv, hg = ag * inv, hb = ab * inv;
        const float hm1 = a1 * inv;
        // second central moment of the bilinear mixture: mean of the taps'
        // central moments plus the spread of their means (no cancellation)
        float s2 = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float d = t1[t] - hm1;
            s2 = ok[t] ? fmaf(bw[t], fmaf(d, d, t2[t]), s2) : s2;
        }
        const float hm2c = s2 * inv;
        // ---- history rectification: variance colour clamp ----
        if (CLAMP) {
            float3 lo, hi;
            box_bounds(tile, lx, ly, a.gamma, lo, hi);
            hr = fminf(fmaxf(hr, lo.x), hi.x);
            hg = fminf(fmaxf(hg, lo.y), hi.y);
            hb = fminf(fmaxf(hb, lo.z), hi.z);
        }
        if (FEAT) {
            float f[SV_MLP_IN] = {L, luma(hr, hg, hb), fmaxf(hm2c, 0.f), box_luma_var(tile, lx, ly),
                                  (float)min(nmax + 1, a.max_hist) / 255.0f,
                                  ldo<T>(a.dzdx, o), ldo<T>(a.dzdy, o), nxc, nyc, nzc,
                                  mv_ok ? sqrtf(fmaf(mvy, mvy, mvx * mvx)) : 0.f,
                                  ldo<T>(a.alr, o), ldo<T>(a.alg, o), ldo<T>(a.alb, o)};
            store_features(a, x, y, f);
            if (a.fhr) {
                stf(a.fhr, o, hr);
                stf(a.fhg, o, hg);
                stf(a.fhb, o, hb);
            }
            return;
        }
        // ---- accumulation ----
        n = min(nmax + 1, a.max_hist);
        const float inv_n = 1.0f / (float)n;
        const float ac = fmaxf(a.alpha_map ? ldf(a.alpha_map, o) : a.alpha, inv_n);
        const float am = fmaxf(a.alpha_m, inv_n);
        outr = fmaf(ac, c.x - hr, hr);
        outg = fmaf(ac, c.y - hg, hg);
        outb = fmaf(ac, c.z - hb, hb);
        const float dl = L - hm1;
        m1 = fmaf(am, dl, hm1);
        // EMA of the raw moments written for the central one:
        // (1 - am) (m2c + am (L - m1)^2)
        m2c = (1.0f - am) * fmaf(am * dl, dl, hm2c);
    }
    sto<T>(a.or_, o, outr);
    sto<T>(a.og, o, outg);
    sto<T>(a.ob, o, outb);
    stf(a.om1, o, m1);
    stf(a.om2c, o, m2c);
    a.on[o] = (uint8_t)n;
}

template <typename T, bool TM, bool CLAMP, bool USE_ID, bool FEAT>
__global__ __launch_bounds__(256) void temporal_k(TemporalArgs a) {
    __shared__ float4 tile[(kTX + 2) * (kTY + 2)];
    const int gxt = (a.w + kTX - 1) / kTX;
    const int t = xcd_tile(gxt * ((a.h + kTY - 1) / kTY));
    if (t < 0) return;
    const int by = t / gxt, bx = t - by * gxt;
    temporal_tile<T, TM, CLAMP, USE_ID, FEAT>(a, tile, bx, by);
}

template <typename T, bool TM, bool CLAMP, bool USE_ID, bool FEAT>
__global__ __launch_bounds__(256) void temporal_batch_k(const TemporalArgs *args, const int *prefix,
                                                        int n, int total) {
    __shared__ float4 tile[(kTX + 2) * (kTY + 2)];
    const int per = (total + kXCD - 1) / kXCD, xcd = (int)blockIdx.x % kXCD;
    for (int slot = (int)blockIdx.x / kXCD; slot < per; slot += (int)gridDim.x / kXCD) {
        const int t = xcd * per + slot;
        if (t >= total) break;
        const int s = batch_stream(prefix, n, t);
        const TemporalArgs a = args[s];
        const int lt = t - prefix[s], gxt = (a.w + kTX - 1) / kTX;
        temporal_tile<T, TM, CLAMP, USE_ID, FEAT>(a, tile, lt % gxt, lt / gxt);
        __syncthreads();  // the next tile's staging reuses the LDS
    }
}

template <typename T, bool TM, bool CLAMP, bool USE_ID, bool FEAT>
static void temporal_batch_launch(const void *args, const int *prefix, int n, int total, int bpc,
                                  hipStream_t s) {
    hipLaunchKernelGGL((temporal_batch_k<T, TM, CLAMP, USE_ID, FEAT>),
                       dim3(batch_grid(total, bpc)), dim3(256), 0, s, (const TemporalArgs *)args,
                       prefix, n, total);
}

struct ClampArgs {
    const void *hr, *hg, *hb, *cr, *cg, *cb, *z;
    void *or_, *og, *ob;
    int w, h, pitch;
    float gamma;
};

template <typename T>
__global__ __launch_bounds__(256) void clamp_k(ClampArgs a) {
    __shared__ float4 tile[(kTX + 2) * (kTY + 2)];
    const int gxt = (a.w + kTX - 1) / kTX;
    const int t = xcd_tile(gxt * ((a.h + kTY - 1) / kTY));
    if (t < 0) return;
    const int by = t / gxt, bx = t - by * gxt;
    stage_current<T, false>(tile, a.cr, a.cg, a.cb, a.z, a.w, a.h, a.pitch, 0.f, bx, by);
    __syncthreads();
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int x = bx * kTX + lx, y = by * kTY + ly;
    if (x >= a.w || y >= a.h) return;
    const uint32_t o = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
    float r = ldo<T>(a.hr, o), g = ldo<T>(a.hg, o), b = ldo<T>(a.hb, o);
    const bool active = a.gamma > 0.f && tile[(ly + 1) * (kTX + 2) + lx + 1].w > 0.f;
    if (active) {
        float3 lo, hi;
        box_bounds(tile, lx, ly, a.gamma, lo, hi);
        r = fminf(fmaxf(r, lo.x), hi.x);
        g = fminf(fmaxf(g, lo.y), hi.y);
        b = fminf(fmaxf(b, lo.z), hi.z);
    }
    sto<T>(a.or_, o, r);
    sto<T>(a.og, o, g);
    sto<T>(a.ob, o, b);
}

template <typename T, bool TM, bool CLAMP, bool USE_ID, bool FEAT>
static void launch_temporal_one(const TemporalArgs &a, dim3 grid, hipStream_t s) {
    const int tiles = ((a.w + kTX - 1) / kTX) * ((a.h + kTY - 1) / kTY);
    if (record_pass(&temporal_batch_launch<T, TM, CLAMP, USE_ID, FEAT>, a, tiles, 8)) return;
    hipLaunchKernelGGL((temporal_k<T, TM, CLAMP, USE_ID, FEAT>), grid, dim3(256), 0, s, a);
}

template <typename T, bool TM, bool CLAMP, bool FEAT>
static void launch_temporal_id(const TemporalArgs &a, bool use_id, dim3 grid, hipStream_t s) {
    if (use_id) launch_temporal_one<T, TM, CLAMP, true, FEAT>(a, grid, s);
    else launch_temporal_one<T, TM, CLAMP, false, FEAT>(a, grid, s);
}

template <typename T, bool FEAT>
static void launch_temporal(const TemporalArgs &a, bool tm, bool clamp, bool use_id, dim3 grid,
                            hipStream_t s) {
    if (tm) {
        if (clamp) launch_temporal_id<T, true, true, FEAT>(a, use_id, grid, s);
        else launch_temporal_id<T, true, false, FEAT>(a, use_id, grid, s);
    } else {
        if (clamp) launch_temporal_id<T, false, true, FEAT>(a, use_id, grid, s);
        else launch_temporal_id<T, false, false, FEAT>(a, use_id, grid, s);
    }
}

}  // namespace sv

extern "C" int sv_temporal(const sv_temporal_io *io, sv_dims d, sv_dtype t,
                           const sv_temporal_params *p, sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    int dc = check_dims(d);
    if (dc < 0 || !io || !p) return SV_EINVAL;
    if (p->max_hist < 1 || p->max_hist > 255) return SV_EINVAL;
    if (dc == 1) return SV_OK;
    const bool use_id = (p->flags & SV_T_USE_ID) != 0;
    const bool clamp = (p->flags & SV_T_CLAMP) != 0 && p->gamma > 0.f;
    const bool tm = (p->flags & SV_T_TONEMAP_IN) != 0;
    const void *req[] = {io->cur.r, io->cur.g, io->cur.b, io->g.z, io->g.nx, io->g.ny, io->g.nz,
                         io->mvx, io->mvy, io->prev.z, io->prev.nx, io->prev.ny, io->prev.nz,
                         io->hist.r, io->hist.g, io->hist.b, io->hist_m1, io->hist_m2c,
                         io->hist_n, io->out.r, io->out.g, io->out.b, io->out_m1,
                         io->out_m2c, io->out_n};
    for (const void *q : req)
        if (!q) return SV_EINVAL;
    if (use_id && (!io->g.id || !io->prev.id)) return SV_EINVAL;
    const size_t es = elem_size(t);
    const span ins[] = {
        plane_span(io->cur.r, d, es), plane_span(io->cur.g, d, es), plane_span(io->cur.b, d, es),
        plane_span(io->g.z, d, es), plane_span(io->g.nx, d, es), plane_span(io->g.ny, d, es),
        plane_span(io->g.nz, d, es), plane_span(io->mvx, d, es), plane_span(io->mvy, d, es),
        plane_span(io->prev.z, d, es), plane_span(io->prev.nx, d, es),
        plane_span(io->prev.ny, d, es), plane_span(io->prev.nz, d, es),
        plane_span(io->hist.r, d, es), plane_span(io->hist.g, d, es),
        plane_span(io->hist.b, d, es), plane_span(io->hist_m1, d, 4),
        plane_span(io->hist_m2c, d, 4), plane_span(io->hist_n, d, 1),
        use_id ? plane_span(io->g.id, d, 1) : span{0, 0},
        use_id ? plane_span(io->prev.id, d, 1) : span{0, 0},
        io->alpha_map ? plane_span(io->alpha_map, d, 4) : span{0, 0}};
    const span outs[] = {plane_span(io->out.r, d, es), plane_span(io->out.g, d, es),
                         plane_span(io->out.b, d, es), plane_span(io->out_m1, d, 4),
                         plane_span(io->out_m2c, d, 4), plane_span(io->out_n, d, 1)};
    for (const span &so : outs) {
        for (const span &si : ins)
            if (overlaps(so, si)) return SV_EALIAS;
    }
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j)
            if (overlaps(outs[i], outs[j])) return SV_EALIAS;
    TemporalArgs a{io->cur.r, io->cur.g, io->cur.b, io->g.z, io->g.nx, io->g.ny, io->g.nz,
                   io->g.id, io->mvx, io->mvy, io->prev.z, io->prev.nx, io->prev.ny,
                   io->prev.nz, io->prev.id, io->hist.r, io->hist.g, io->hist.b, io->hist_m1,
                   io->hist_m2c, io->hist_n, io->out.r, io->out.g, io->out.b, io->out_m1,
                   io->out_m2c, io->out_n, io->alpha_map, d.w, d.h, d.pitch, p->alpha,
                   p->alpha_m, p->gamma, p->tau_z, p->tau_n, p->tm_k, p->max_hist};
    dim3 grid(xcd_grid(((d.w + kTX - 1) / kTX) * ((d.h + kTY - 1) / kTY)));
    hipStream_t s = as_stream(stream);
    if (t == SV_F32) launch_temporal<float, false>(a, tm, clamp, use_id, grid, s);
    else launch_temporal<half_t, false>(a, tm, clamp, use_id, grid, s);
    return hip_status(hipGetLastError());
}

extern "C" int sv_mlp_features(const sv_temporal_io *io, const sv_rgb *albedo, const sv_mlp *w,
                               void *feat, const sv_rgb *hist_out, sv_dims d, sv_dtype t,
                               const sv_temporal_params *p, sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    int dc = check_dims(d);
    if (dc < 0 || !io || !p || !albedo || !w) return SV_EINVAL;
    if (p->max_hist < 1 || p->max_hist > 255) return SV_EINVAL;
    if (dc == 1) return SV_OK;
    const bool use_id = (p->flags & SV_T_USE_ID) != 0;
    const bool clamp = (p->flags & SV_T_CLAMP) != 0 && p->gamma > 0.f;
    const bool tm = (p->flags & SV_T_TONEMAP_IN) != 0;
    const void *req[] = {io->cur.r, io->cur.g, io->cur.b, io->g.z, io->g.dzdx, io->g.dzdy,
                         io->g.nx, io->g.ny, io->g.nz, io->mvx, io->mvy, io->prev.z,
                         io->prev.nx, io->prev.ny, io->prev.nz, io->hist.r, io->hist.g,
                         io->hist.b, io->hist_m1, io->hist_m2c, io->hist_n, albedo->r,
                         albedo->g, albedo->b, feat, w->mu, w->inv_s};
    for (const void *q : req)
        if (!q) return SV_EINVAL;
    if (((uintptr_t)feat & 15u) != 0) return SV_EINVAL;
    if (use_id && (!io->g.id || !io->prev.id)) return SV_EINVAL;
    if (hist_out && (!hist_out->r || !hist_out->g || !hist_out->b)) return SV_EINVAL;
    const size_t es = elem_size(t);
    const span fs{(uintptr_t)feat, (uintptr_t)feat + (size_t)d.w * (size_t)d.h * 32u};
    const span ins[] = {
        plane_span(io->cur.r, d, es), plane_span(io->cur.g, d, es), plane_span(io->cur.b, d, es),
        plane_span(io->g.z, d, es), plane_span(io->g.dzdx, d, es), plane_span(io->g.dzdy, d, es),
        plane_span(io->g.nx, d, es), plane_span(io->g.ny, d, es), plane_span(io->g.nz, d, es),
        plane_span(io->mvx, d, es), plane_span(io->mvy, d, es), plane_span(io->prev.z, d, es),
        plane_span(io->prev.nx, d, es), plane_span(io->prev.ny, d, es),
        plane_span(io->prev.nz, d, es), plane_span(io->hist.r, d, es),
        plane_span(io->hist.g, d, es), plane_span(io->hist.b, d, es),
        plane_span(io->hist_m1, d, 4), plane_span(io->hist_m2c, d, 4),
        plane_span(io->hist_n, d, 1), plane_span(albedo->r, d, es), plane_span(albedo->g, d, es),
        plane_span(albedo->b, d, es),
        use_id ? plane_span(io->g.id, d, 1) : span{0, 0},
        use_id ? plane_span(io->prev.id, d, 1) : span{0, 0}};
    span outs[4] = {fs, span{0, 0}, span{0, 0}, span{0, 0}};
    if (hist_out) {
        outs[1] = plane_span(hist_out->r, d, 4);
        outs[2] = plane_span(hist_out->g, d, 4);
        outs[3] = plane_span(hist_out->b, d, 4);
    }
    for (const span &so : outs) {
        for (const span &si : ins)
            if (overlaps(so, si)) return SV_EALIAS;
    }
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j)
            if (overlaps(outs[i], outs[j])) return SV_EALIAS;
    TemporalArgs a{io->cur.r, io->cur.g, io->cur.b, io->g.z, io->g.nx, io->g.ny, io->g.nz,
                   io->g.id, io->mvx, io->mvy, io->prev.z, io->prev.nx, io->prev.ny,
                   io->prev.nz, io->prev.id, io->hist.r, io->hist.g, io->hist.b, io->hist_m1,
                   io->hist_m2c, io->hist_n, nullptr, nullptr, nullptr, nullptr,
                   nullptr, nullptr, nullptr, d.w, d.h, d.pitch, p->alpha,
                   p->alpha_m, p->gamma, p->tau_z, p->tau_n, p->tm_k, p->max_hist,
                   io->g.dzdx, io->g.dzdy, albedo->r, albedo->g, albedo->b, (uint4 *)feat,
                   hist_out ? (float *)hist_out->r : nullptr,
                   hist_out ? (float *)hist_out->g : nullptr,
                   hist_out ? (float *)hist_out->b : nullptr, w->mu, w->inv_s};
    dim3 grid(xcd_grid(((d.w + kTX - 1) / kTX) * ((d.h + kTY - 1) / kTY)));
    hipStream_t s = as_stream(stream);
    if (t == SV_F32) launch_temporal<float, true>(a, tm, clamp, use_id, grid, s);
    else launch_temporal<half_t, true>(a, tm, clamp, use_id, grid, s);
    return hip_status(hipGetLastError());
}

extern "C" int sv_clamp(const sv_rgb *hist, const sv_rgb *cur, const sv_rgb *out, const void *z,
                        sv_dims d, sv_dtype t, float gamma, sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    int dc = check_dims(d);
    if (dc < 0 || !hist || !cur || !out) return SV_EINVAL;
    if (dc == 1) return SV_OK;
    if (!hist->r || !hist->g || !hist->b || !cur->r || !cur->g || !cur->b || !out->r ||
        !out->g || !out->b)
        return SV_EINVAL;
    const size_t es = elem_size(t);
    const span ins[] = {plane_span(cur->r, d, es), plane_span(cur->g, d, es),
                        plane_span(cur->b, d, es), z ? plane_span(z, d, es) : span{0, 0}};
    const span outs[] = {plane_span(out->r, d, es), plane_span(out->g, d, es),
                         plane_span(out->b, d, es)};
    for (const span &so : outs)
        for (const span &si : ins)
            if (overlaps(so, si)) return SV_EALIAS;
    ClampArgs a{hist->r, hist->g, hist->b, cur->r, cur->g, cur->b, z,
                out->r, out->g, out->b, d.w, d.h, d.pitch, gamma};
    dim3 grid(xcd_grid(((d.w + kTX - 1) / kTX) * ((d.h + kTY - 1) / kTY)));
    if (t == SV_F32)
        hipLaunchKernelGGL(clamp_k<float>, grid, dim3(256), 0, as_stream(stream), a);
    else
        hipLaunchKernelGGL(clamp_k<half_t>, grid, dim3(256), 0, as_stream(stream), a);
    return hip_status(hipGetLastError());
}
