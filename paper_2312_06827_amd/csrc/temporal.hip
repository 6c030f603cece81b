// Temporal filter: backward reprojection of the history, variance colour
// clamp of the reprojected colour, and accumulation of colour and luminance
// moments (Section 2; Section 3 step 4; Section 3.1).  One fused pass:
// every pixel reads its current colour (tone mapped on the fly), its 3x3
// neighbourhood through an LDS tile, and four bilinear history taps.
#include "mlp_impl.h"

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
    int tm;  // forward tone map of the current colour (a uniform branch)
    // feature mode only
    const void *dzdx, *dzdy, *alr, *alg, *alb;
    uint4 *feat;              // two 16-byte halves per pixel, row y * w + x
    float *fhr, *fhg, *fhb;   // clamped reprojected history (optional)
    const float *mu, *inv_s;  // standardisation
    // learned mode only
    const float *mparams;
    const uint16_t *mwq;
    float *kappa_out, *alpha_out;
    // variance, first part
    float *var_out;
    VarWork *var_work;
    uint32_t var_cap;
    int min_hist;
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

// History rectification: none, the per-channel variance colour clamp, or
// variance colour clipping toward the box centre.
enum { kRectOff = 0, kRectClamp = 1, kRectClip = 2 };

// 3x3 box of the tile around (lx+1, ly+1): centre mu and half-widths
// gamma sigma per channel from the mean and population variance over valid
// entries (w component 1, else 0; their colour is masked out here).
// Binary64: the clamp bounds mu -+ gamma sigma are differences of
// quantities of the colour's size and may be close to zero, where binary32
// bounds would carry errors far above their own size (measured: 1.6e-5
// relative on random colours, 1.3e-4 on binary visibility); clipping
// divides by the history's distance from mu.  One pass of sums of x and
// x^2 suffices there:
// products of binary32 values are exact in binary64, and the cancellation
// in E[x^2] - E[x]^2 costs at most log2(mu^2 / sigma^2) of its 53 bits.
__device__ __forceinline__ void box_stats(const float4 *tile, int lx, int ly, float gamma,
                                          double3 &mu, double3 &half) {
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
    mu = make_double3(mr, mg, mb);
    half = make_double3(gamma * sqrt(vr), gamma * sqrt(vg), gamma * sqrt(vb));
}

// Rectifies the history colour (r, g, b) against the box of (lx+1, ly+1).
// Clamp: each channel to [mu - gamma sigma, mu + gamma sigma].  Clip: a
// colour outside the box moves toward mu along the segment from mu onto the
// box's surface, mu + t (h - mu) with t the smallest ratio half / |h - mu|
// over the channels outside (so a channel with zero spread and a nonzero
// deviation gives mu); a colour inside is kept as it is.
template <int RECT>
__device__ __forceinline__ void rectify(const float4 *tile, int lx, int ly, float gamma, float &r,
                                        float &g, float &b) {
    if (RECT == kRectOff) return;
    double3 mu, e;
    box_stats(tile, lx, ly, gamma, mu, e);
    if (RECT == kRectClamp) {
        r = fminf(fmaxf(r, (float)(mu.x - e.x)), (float)(mu.x + e.x));
        g = fminf(fmaxf(g, (float)(mu.y - e.y)), (float)(mu.y + e.y));
        b = fminf(fmaxf(b, (float)(mu.z - e.z)), (float)(mu.z + e.z));
        return;
    }
    const double dr = (double)r - mu.x, dg = (double)g - mu.y, db = (double)b - mu.z;
    const double ar = fabs(dr), ag = fabs(dg), ab = fabs(db);
    double t = 1.0;
    if (ar > e.x) t = fmin(t, e.x / ar);
    if (ag > e.y) t = fmin(t, e.y / ag);
    if (ab > e.z) t = fmin(t, e.z / ab);
    if (t < 1.0) {
        r = (float)fma(t, dr, mu.x);
        g = (float)fma(t, dg, mu.y);
        b = (float)fma(t, db, mu.z);
    }
}

// Stage the current colour (tone mapped if tm) of the tile and a one-pixel
// apron; w = 1 for pixels inside the image that are not empty, else 0.
template <typename T>
__device__ __forceinline__ void stage_current(float4 *tile, const void *cr, const void *cg,
                                              const void *cb, const void *zp, int w, int h,
                                              int pitch, bool tm, float tm_k, int bx, int by) {
    // unrolled, every load issued from an in-image address (masked after)
    const int x0 = (int)bx * kTX - 1, y0 = (int)by * kTY - 1;
    constexpr int NS = (kTX + 2) * (kTY + 2), IT = (NS + 255) / 256;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = threadIdx.x + it * 256;
        const int r = i / (kTX + 2), c = i - r * (kTX + 2);
        const int gx = x0 + c, gy = y0 + r;
        const bool in = i < NS && gx >= 0 && gx < w && gy >= 0 && gy < h;
        const uint32_t o = vofs(in ? (uint32_t)gy * (uint32_t)pitch + (uint32_t)gx : 0u);
        float R = ldo<T>(cr, o), G = ldo<T>(cg, o), B = ldo<T>(cb, o);
        const float zz = zp ? ldo<T>(zp, o) : 1.f;
        if (tm) {
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

// Standardise the 14 raw features and pack them as 16 bfloat16 (the last
// two zero) into eight words.
__device__ __forceinline__ void standardise_pack(const TemporalArgs &a, const float (&f)[SV_MLP_IN],
                                                 uint32_t (&pk)[8]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k0 = 2 * i, k1 = 2 * i + 1;
        // features 14 and 15 are the zero pads
        const uint32_t lo = k0 < SV_MLP_IN ? to_bf16((f[k0] - a.mu[k0]) * a.inv_s[k0]) : 0u;
        const uint32_t hi = k1 < SV_MLP_IN ? to_bf16((f[k1] - a.mu[k1]) * a.inv_s[k1]) : 0u;
        pk[i] = lo | (hi << 16);
    }
}

// The pixel's 32-byte feature row.
__device__ __forceinline__ void store_features(const TemporalArgs &a, int x, int y,
                                               const float (&f)[SV_MLP_IN]) {
    uint32_t pk[8];
    standardise_pack(a, f, pk);
    uint4 *row = a.feat + 2 * ((size_t)y * (size_t)a.w + (size_t)x);
    row[0] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
    row[1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
}

// What one pixel's reprojection and clamp yield (before the blend).
struct PxState {
    float4 c;  // current colour (tone mapped); w: in the image and not empty
    float L, zc, nxc, nyc, nzc, mvx, mvy;
    uint32_t o;
    bool inimg, empty, mv_ok, any;
    float hr, hg, hb, hm1, hm2c;  // reprojected history, clamped (valid if any)
    int nmax;
};

// Everything one pixel reads from memory (its own G-buffer and motion, and
// the four bilinear history taps), gathered before the tile's barrier so
// that these loads overlap the staging of the current colour.
struct PxLoads {
    float zc, nxc, nyc, nzc, mvx, mvy;
    int idc;
    float bw[4], tz[4], tnx[4], tny[4], tnz[4], tr[4], tg[4], tb[4], t1[4], t2[4];
    int thn[4], tid_[4];
    bool inb[4];
    bool mv_ok;
};

template <typename T, bool USE_ID>
__device__ __forceinline__ void px_gather(const TemporalArgs &a, int x, int y, PxLoads &g) {
    const bool inimg = x < a.w && y < a.h;
    const uint32_t o = vofs(inimg ? (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x : 0u);
    g.zc = ldo<T>(a.z, o);
    g.nxc = ldo<T>(a.nx, o);
    g.nyc = ldo<T>(a.ny, o);
    g.nzc = ldo<T>(a.nz, o);
    g.mvx = ldo<T>(a.mvx, o);
    g.mvy = ldo<T>(a.mvy, o);
    g.idc = USE_ID ? a.id[o] : 0;
    // ---- backward reprojection: bilinear taps around p + mv ----
    // Every load of the four taps is issued before any test, so the taps'
    // memory latencies overlap instead of chaining through the tests.
    const float mvx = g.mvx, mvy = g.mvy;
    const bool mv_ok = fabsf(mvx) < 1048576.0f && fabsf(mvy) < 1048576.0f;
    g.mv_ok = mv_ok;
    const float fx0 = mv_ok ? floorf(mvx) : 0.f, fy0 = mv_ok ? floorf(mvy) : 0.f;
    // The bilinear factors of the far and near taps, each formed from mv:
    // f = mv - floor(mv) and e = (floor(mv) + 1) - mv.  Whichever of the two
    // is below 1/2 is exact in binary32 (Sterbenz), the other within an ulp.
    // e = 1 - f would not do: for -1/2 < mv < 0, f = 1 + mv rounds, and a
    // tiny 1 - f then carries a large relative error, which matters where
    // the near taps are the only usable ones.
    const float fx = mvx - fx0, fy = mvy - fy0;
    const float ex = (fx0 + 1.0f) - mvx, ey = (fy0 + 1.0f) - mvy;
    const int x0 = x + (int)fx0, y0 = y + (int)fy0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int tx = x0 + (t & 1), ty = y0 + (t >> 1);
        const float wx = (t & 1) ? fx : ex, wy = (t >> 1) ? fy : ey;
        g.bw[t] = wx * wy;
        // a nonzero weight, decided on the factors (their product could
        // underflow where the exact one does not)
        g.inb[t] = inimg && mv_ok && wx > 0.f && wy > 0.f && tx >= 0 && tx < a.w && ty >= 0 &&
                   ty < a.h;
        const uint32_t q = vofs(g.inb[t] ? (uint32_t)ty * (uint32_t)a.pitch + (uint32_t)tx : o);
        g.thn[t] = a.hn[q];
        g.tz[t] = ldo<T>(a.pz, q);
        g.tnx[t] = ldo<T>(a.pnx, q);
        g.tny[t] = ldo<T>(a.pny, q);
        g.tnz[t] = ldo<T>(a.pnz, q);
        g.tid_[t] = USE_ID ? a.pid[q] : 0;
        g.tr[t] = ldo<T>(a.hr, q);
        g.tg[t] = ldo<T>(a.hg, q);
        g.tb[t] = ldo<T>(a.hb, q);
        g.t1[t] = ldf(a.hm1, q);
        g.t2[t] = ldf(a.hm2c, q);
    }
}

// The validity tests, the renormalised history, its central moment and the
// clamp, from the gathered loads and the staged tile.
template <int RECT, bool USE_ID>
__device__ __forceinline__ PxState px_reproject(const TemporalArgs &a, const float4 *tile, int lx,
                                                int ly, int x, int y, const PxLoads &g) {
    PxState s;
    s.inimg = x < a.w && y < a.h;
    s.o = vofs(s.inimg ? (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x : 0u);
    s.c = tile[(ly + 1) * (kTX + 2) + lx + 1];
    s.L = luma(s.c.x, s.c.y, s.c.z);
    s.zc = g.zc;
    s.empty = !s.inimg || empty_px(s.zc);
    s.any = false;
    s.mv_ok = false;
    s.nxc = s.nyc = s.nzc = s.mvx = s.mvy = 0.f;
    s.hr = s.hg = s.hb = s.hm1 = s.hm2c = 0.f;
    s.nmax = 0;
    if (s.empty) return s;
    const float zc = s.zc, nxc = g.nxc, nyc = g.nyc, nzc = g.nzc;
    s.nxc = nxc;
    s.nyc = nyc;
    s.nzc = nzc;
    s.mvx = g.mvx;
    s.mvy = g.mvy;
    s.mv_ok = g.mv_ok;
    float sw = 0.f, ar = 0.f, ag = 0.f, ab = 0.f, a1 = 0.f;
    int nmax = 0;
    bool ok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        ok[t] = g.inb[t] && g.thn[t] >= 1 && depth_consistent(g.tz[t], zc, a.tau_z) &&
                normal_consistent(g.tnx[t], g.tny[t], g.tnz[t], nxc, nyc, nzc, a.tau_n) &&
                (!USE_ID || g.tid_[t] == g.idc);
        // selects, not zero weights: an unusable tap's history may hold
        // anything (even NaN) and must not reach the sums
        sw = ok[t] ? sw + g.bw[t] : sw;
        ar = ok[t] ? fmaf(g.bw[t], g.tr[t], ar) : ar;
        ag = ok[t] ? fmaf(g.bw[t], g.tg[t], ag) : ag;
        ab = ok[t] ? fmaf(g.bw[t], g.tb[t], ab) : ab;
        a1 = ok[t] ? fmaf(g.bw[t], g.t1[t], a1) : a1;
        nmax = ok[t] ? max(nmax, g.thn[t]) : nmax;
    }
    s.any = ok[0] || ok[1] || ok[2] || ok[3];
    s.nmax = nmax;
    if (!s.any) return s;
    const float inv = 1.0f / sw;
    float hr = quot(ar, sw, inv), hg = quot(ag, sw, inv), hb = quot(ab, sw, inv);
    const float hm1 = quot(a1, sw, inv);
    // second central moment of the bilinear mixture: mean of the taps'
    // central moments plus the spread of their means (no cancellation)
    float s2 = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float d = g.t1[t] - hm1;
        s2 = ok[t] ? fmaf(g.bw[t], fmaf(d, d, g.t2[t]), s2) : s2;
    }
    // ---- history rectification: variance colour clamp or clip ----
    rectify<RECT>(tile, lx, ly, a.gamma, hr, hg, hb);
    s.hr = hr;
    s.hg = hg;
    s.hb = hb;
    s.hm1 = hm1;
    s.hm2c = s2 * inv;
    return s;
}

// The 14 raw features of the learned component (all zero for an empty
// pixel or one outside the image).
template <typename T>
__device__ __forceinline__ void px_features(const TemporalArgs &a, const float4 *tile, int lx,
                                            int ly, const PxState &s, float (&f)[SV_MLP_IN]) {
    if (s.empty) {
#pragma unroll
        for (int i = 0; i < SV_MLP_IN; ++i) f[i] = 0.f;
        return;
    }
    const uint32_t o = s.o;
    f[0] = s.L;
    f[1] = s.any ? luma(s.hr, s.hg, s.hb) : 0.f;
    f[2] = s.any ? fmaxf(s.hm2c, 0.f) : 0.f;
    f[3] = box_luma_var(tile, lx, ly);
    f[4] = s.any ? (float)min(s.nmax + 1, a.max_hist) / 255.0f : 1.0f / 255.0f;
    f[5] = ldo<T>(a.dzdx, o);
    f[6] = ldo<T>(a.dzdy, o);
    f[7] = s.nxc;
    f[8] = s.nyc;
    f[9] = s.nzc;
    f[10] = s.mv_ok ? sqrtf(fmaf(s.mvy, s.mvy, s.mvx * s.mvx)) : 0.f;
    f[11] = ldo<T>(a.alr, o);
    f[12] = ldo<T>(a.alg, o);
    f[13] = ldo<T>(a.alb, o);
}

// Blend colour and moments (alpha: the colour blend factor before the 1/n
// floor) and store the pixel's outputs.
template <typename T>
__device__ __forceinline__ void px_blend(const TemporalArgs &a, const PxState &s, float alpha,
                                         int &n_out, float &m2c_out) {
    const uint32_t o = s.o;
    n_out = 0;
    m2c_out = 0.f;
    if (s.empty) {
        sto<T>(a.or_, o, s.c.x);
        sto<T>(a.og, o, s.c.y);
        sto<T>(a.ob, o, s.c.z);
        stf(a.om1, o, 0.f);
        stf(a.om2c, o, 0.f);
        a.on[o] = 0;
        return;
    }
    float outr, outg, outb, m1, m2c;
    int n;
    if (!s.any) {
        outr = s.c.x;
        outg = s.c.y;
        outb = s.c.z;
        m1 = s.L;
        m2c = 0.f;
        n = 1;
    } else {
        // ---- accumulation ----
        n = min(s.nmax + 1, a.max_hist);
        const float inv_n = 1.0f / (float)n;
        const float ac = fmaxf(alpha, inv_n);
        const float am = fmaxf(a.alpha_m, inv_n);
        outr = fmaf(ac, s.c.x - s.hr, s.hr);
        outg = fmaf(ac, s.c.y - s.hg, s.hg);
        outb = fmaf(ac, s.c.z - s.hb, s.hb);
        const float dl = s.L - s.hm1;
        m1 = fmaf(am, dl, s.hm1);
        // EMA of the raw moments written for the central one:
        // (1 - am) (m2c + am (L - m1)^2)
        m2c = (1.0f - am) * fmaf(am * dl, dl, s.hm2c);
    }
    sto<T>(a.or_, o, outr);
    sto<T>(a.og, o, outg);
    sto<T>(a.ob, o, outb);
    stf(a.om1, o, m1);
    stf(a.om2c, o, m2c);
    a.on[o] = (uint8_t)n;
    n_out = n;
    m2c_out = m2c;
}

// The network on this workgroup's 256 pixels: every lane's standardised
// features go through LDS into the matrix operands of its wave's two
// 32-pixel blocks; returns this lane's alpha and kappa.  Every thread of
// the workgroup must call it (barrier and matrix instructions).
// The network's parameters come from the workgroup's LDS copy (`ns`: this
// thread's share of it, loaded earlier): the pass is bound by its load path,
// which per-lane weight loads would add to.
__device__ __forceinline__ void px_network(const TemporalArgs &a, uint4 *s_feat, uint16_t *s_w,
                                           float *s_b, const NetStage &ns,
                                           const float (&f)[SV_MLP_IN], float &alpha,
                                           float &kappa) {
    uint32_t pk[8];
    standardise_pack(a, f, pk);
    s_feat[2 * threadIdx.x] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
    s_feat[2 * threadIdx.x + 1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
    net_store(ns, s_w, s_b);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 31, hf = lane >> 5;
    float o0 = 0.f, o1 = 0.f;
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        const uint2 *row = (const uint2 *)(s_feat + 2 * (wave * 64 + blk * 32 + col));
        bf16x4 x[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const uint2 v = row[2 * kb + hf];
            x[kb][0] = (short)(v.x & 0xFFFFu);
            x[kb][1] = (short)(v.x >> 16);
            x[kb][2] = (short)(v.y & 0xFFFFu);
            x[kb][3] = (short)(v.y >> 16);
        }
        FwdOut r;
        forward_block_lds(s_w, s_b, col, hf, x, r);
        // lanes l and l + 32 both hold pixel blk * 32 + l % 32's outputs:
        // lane l keeps the block that contains its own pixel (blk == l / 32)
        if (blk == hf) {
            o0 = r.o0;
            o1 = r.o1;
        }
    }
    mlp_heads(o0, o1, alpha, kappa);
}

// One 64x4 tile (bx, by).  MODE: kBlend (the temporal step), kFeat
// (feature rows instead of the blend) or kLearn (features, the network,
// then the blend with the network's alpha; kappa written out).  Returns
// once this thread's pixel is done (the caller's barrier follows).
enum { kBlend = 0, kFeat = 1, kLearn = 2 };

template <typename T, int RECT, bool USE_ID, int MODE>
__device__ __forceinline__ void temporal_tile(const TemporalArgs &a, float4 *tile, uint4 *s_feat,
                                              uint16_t *s_w, float *s_b, uint32_t *wave_n,
                                              uint32_t &base_sh, int bx, int by) {
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int x = bx * kTX + lx, y = by * kTY + ly;
    PxLoads g;
    px_gather<T, USE_ID>(a, x, y, g);
    stage_current<T>(tile, a.cr, a.cg, a.cb, a.z, a.w, a.h, a.pitch, a.tm != 0, a.tm_k, bx, by);
    __syncthreads();
    const PxState s = px_reproject<RECT, USE_ID>(a, tile, lx, ly, x, y, g);
    if (MODE == kFeat) {
        if (!s.inimg) return;
        float f[SV_MLP_IN];
        px_features<T>(a, tile, lx, ly, s, f);
        store_features(a, x, y, f);
        if (a.fhr) {
            stf(a.fhr, s.o, s.any ? s.hr : 0.f);
            stf(a.fhg, s.o, s.any ? s.hg : 0.f);
            stf(a.fhb, s.o, s.any ? s.hb : 0.f);
        }
        return;
    }
    float alpha = a.alpha;
    if (MODE == kLearn) {
        NetStage ns;
        net_issue(a.mparams, a.mwq, ns);  // in flight while the features are formed
        float f[SV_MLP_IN], kappa;
        px_features<T>(a, tile, lx, ly, s, f);
        px_network(a, s_feat, s_w, s_b, ns, f, alpha, kappa);
        if (s.inimg && a.kappa_out) stf(a.kappa_out, s.o, kappa);
        if (s.inimg && a.alpha_out) stf(a.alpha_out, s.o, alpha);
    } else if (a.alpha_map && s.inimg && s.any) {
        alpha = ldf(a.alpha_map, s.o);
    }
    int n = 0;
    float m2c = 0.f;
    if (s.inimg) px_blend<T>(a, s, alpha, n, m2c);
    if (a.var_out) {  // the variance estimate's first part (uniform branch)
        const bool live = s.inimg && !s.empty;
        const bool spatial = live && n < a.min_hist;
        if (s.inimg && !spatial) stf(a.var_out, s.o, live ? fmaxf(0.f, m2c) : 0.f);
        const int gxt = (a.w + kTX - 1) / kTX;
        list_short_pixel(a.var_work, a.var_cap, by * gxt + bx, spatial, x, y, wave_n, base_sh);
    }
}

// The learned mode holds the network's matrix accumulators beside the pass's
// own state: it is asked for four waves per SIMD, which it reaches without
// spilling (left alone, its accumulation registers cost it a wave).
#define SV_TEMPORAL_WAVES(MODE) amdgpu_waves_per_eu((MODE) == kLearn ? 4 : 1)

template <typename T, int RECT, bool USE_ID, int MODE>
__global__ __launch_bounds__(256) __attribute__((SV_TEMPORAL_WAVES(MODE))) void temporal_k(
    TemporalArgs a) {
    __shared__ float4 tile[(kTX + 2) * (kTY + 2)];
    __shared__ uint4 s_feat[MODE == kLearn ? 2 * 256 : 1];
    __shared__ uint16_t s_w[MODE == kLearn ? SV_MLP_PARAMS : 1];
    __shared__ float s_b[MODE == kLearn ? kNetBiases : 1];
    __shared__ uint32_t wave_n[4], base_sh;
    const int gxt = (a.w + kTX - 1) / kTX;
    const int t = xcd_tile(gxt * ((a.h + kTY - 1) / kTY));
    if (t < 0) return;
    const int by = t / gxt, bx = t - by * gxt;
    temporal_tile<T, RECT, USE_ID, MODE>(a, tile, s_feat, s_w, s_b, wave_n, base_sh, bx, by);
}

template <typename T, int RECT, bool USE_ID, int MODE>
__global__ __launch_bounds__(256) __attribute__((SV_TEMPORAL_WAVES(MODE))) void temporal_batch_k(
    const TemporalArgs *args, const int *prefix, int n, int total) {
    __shared__ float4 tile[(kTX + 2) * (kTY + 2)];
    __shared__ uint4 s_feat[MODE == kLearn ? 2 * 256 : 1];
    __shared__ uint16_t s_w[MODE == kLearn ? SV_MLP_PARAMS : 1];
    __shared__ float s_b[MODE == kLearn ? kNetBiases : 1];
    __shared__ uint32_t wave_n[4], base_sh;
    int s = 0;
    const int lt = batch_tile(prefix, n, total, s);
    if (lt < 0) return;
    const TemporalArgs a = args[s];  // a copy: the kernel's stores cannot alias it
    const int gxt = (a.w + kTX - 1) / kTX;
    temporal_tile<T, RECT, USE_ID, MODE>(a, tile, s_feat, s_w, s_b, wave_n, base_sh, lt % gxt,
                                         lt / gxt);
}

template <typename T, int RECT, bool USE_ID, int MODE>
static void temporal_batch_launch(const void *args, const int *prefix, int n, int total,
                                  hipStream_t s) {
    hipLaunchKernelGGL((temporal_batch_k<T, RECT, USE_ID, MODE>), dim3(xcd_grid(total)),
                       dim3(256), 0, s, (const TemporalArgs *)args, prefix, n, total);
}

struct ClampArgs {
    const void *hr, *hg, *hb, *cr, *cg, *cb, *z;
    void *or_, *og, *ob;
    int w, h, pitch;
    float gamma;
};

template <typename T, int RECT>
__global__ __launch_bounds__(256) void clamp_k(ClampArgs a) {
    __shared__ float4 tile[(kTX + 2) * (kTY + 2)];
    const int gxt = (a.w + kTX - 1) / kTX;
    const int t = xcd_tile(gxt * ((a.h + kTY - 1) / kTY));
    if (t < 0) return;
    const int by = t / gxt, bx = t - by * gxt;
    stage_current<T>(tile, a.cr, a.cg, a.cb, a.z, a.w, a.h, a.pitch, false, 0.f, bx, by);
    __syncthreads();
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int x = bx * kTX + lx, y = by * kTY + ly;
    if (x >= a.w || y >= a.h) return;
    const uint32_t o = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
    float r = ldo<T>(a.hr, o), g = ldo<T>(a.hg, o), b = ldo<T>(a.hb, o);
    const bool active = a.gamma > 0.f && tile[(ly + 1) * (kTX + 2) + lx + 1].w > 0.f;
    if (active) rectify<RECT>(tile, lx, ly, a.gamma, r, g, b);
    sto<T>(a.or_, o, r);
    sto<T>(a.og, o, g);
    sto<T>(a.ob, o, b);
}

template <typename T, int RECT, bool USE_ID, int MODE>
static void launch_temporal_one(const TemporalArgs &a, dim3 grid, hipStream_t s) {
    const int tiles = ((a.w + kTX - 1) / kTX) * ((a.h + kTY - 1) / kTY);
    if (record_pass(&temporal_batch_launch<T, RECT, USE_ID, MODE>, a, tiles)) return;
    hipLaunchKernelGGL((temporal_k<T, RECT, USE_ID, MODE>), grid, dim3(256), 0, s, a);
}

template <typename T, int RECT, int MODE>
static void launch_temporal_id(const TemporalArgs &a, bool use_id, dim3 grid, hipStream_t s) {
    if (use_id) launch_temporal_one<T, RECT, true, MODE>(a, grid, s);
    else launch_temporal_one<T, RECT, false, MODE>(a, grid, s);
}

template <typename T, int MODE>
static void launch_temporal(const TemporalArgs &a, int rect, bool use_id, dim3 grid,
                            hipStream_t s) {
    if (rect == kRectClip) launch_temporal_id<T, kRectClip, MODE>(a, use_id, grid, s);
    else if (rect == kRectClamp) launch_temporal_id<T, kRectClamp, MODE>(a, use_id, grid, s);
    else launch_temporal_id<T, kRectOff, MODE>(a, use_id, grid, s);
}

// Rectification mode of the temporal flags; -1 when both are set.
static int rect_mode(const sv_temporal_params *p) {
    const bool clamp = (p->flags & SV_T_CLAMP) != 0, clip = (p->flags & SV_T_CLIP) != 0;
    if (clamp && clip) return -1;
    if (!(p->gamma > 0.f)) return kRectOff;
    return clip ? kRectClip : clamp ? kRectClamp : kRectOff;
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
    const int rect = rect_mode(p);
    if (rect < 0) return SV_EINVAL;
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
    if (io->var) {
        if (!io->var_work || io->var_min_hist < 0) return SV_EINVAL;
        const span vs = plane_span(io->var, d, 4);
        const span ws{(uintptr_t)io->var_work,
                      (uintptr_t)io->var_work + sv_variance_work_bytes(d)};
        for (const span &si : ins)
            if (overlaps(vs, si) || overlaps(ws, si)) return SV_EALIAS;
        for (const span &so : outs)
            if (overlaps(vs, so) || overlaps(ws, so)) return SV_EALIAS;
        if (overlaps(vs, ws)) return SV_EALIAS;
    }
    const bool learn = io->mlp != nullptr;
    if (learn) {
        const void *lreq[] = {io->g.dzdx, io->g.dzdy, io->albedo.r, io->albedo.g, io->albedo.b,
                              io->mlp->params, io->mlp->wq, io->mlp->mu, io->mlp->inv_s};
        for (const void *q : lreq)
            if (!q) return SV_EINVAL;
        const span lins[] = {plane_span(io->g.dzdx, d, es), plane_span(io->g.dzdy, d, es),
                             plane_span(io->albedo.r, d, es), plane_span(io->albedo.g, d, es),
                             plane_span(io->albedo.b, d, es)};
        const span louts[] = {io->kappa_out ? plane_span(io->kappa_out, d, 4) : span{0, 0},
                              io->alpha_out ? plane_span(io->alpha_out, d, 4) : span{0, 0}};
        for (const span &so : louts) {
            for (const span &si : ins)
                if (overlaps(so, si)) return SV_EALIAS;
            for (const span &si : lins)
                if (overlaps(so, si)) return SV_EALIAS;
            for (const span &si : outs)
                if (overlaps(so, si)) return SV_EALIAS;
        }
        if (overlaps(louts[0], louts[1])) return SV_EALIAS;
        for (const span &so : outs)
            for (const span &si : lins)
                if (overlaps(so, si)) return SV_EALIAS;
    }
    TemporalArgs a{io->cur.r, io->cur.g, io->cur.b, io->g.z, io->g.nx, io->g.ny, io->g.nz,
                   io->g.id, io->mvx, io->mvy, io->prev.z, io->prev.nx, io->prev.ny,
                   io->prev.nz, io->prev.id, io->hist.r, io->hist.g, io->hist.b, io->hist_m1,
                   io->hist_m2c, io->hist_n, io->out.r, io->out.g, io->out.b, io->out_m1,
                   io->out_m2c, io->out_n, learn ? nullptr : io->alpha_map, d.w, d.h, d.pitch,
                   p->alpha, p->alpha_m, p->gamma, p->tau_z, p->tau_n, p->tm_k, p->max_hist,
                   tm ? 1 : 0};
    dim3 grid(xcd_grid(((d.w + kTX - 1) / kTX) * ((d.h + kTY - 1) / kTY)));
    hipStream_t s = as_stream(stream);
    if (io->var) {
        a.var_out = io->var;
        a.var_work = (VarWork *)io->var_work;
        a.var_cap = (point_grid(d) / kXCD) * 256u;
        a.min_hist = io->var_min_hist;
    }
    if (learn) {
        a.dzdx = io->g.dzdx;
        a.dzdy = io->g.dzdy;
        a.alr = io->albedo.r;
        a.alg = io->albedo.g;
        a.alb = io->albedo.b;
        a.mu = io->mlp->mu;
        a.inv_s = io->mlp->inv_s;
        a.mparams = io->mlp->params;
        a.mwq = io->mlp->wq;
        a.kappa_out = io->kappa_out;
        a.alpha_out = io->alpha_out;
        if (t == SV_F32) launch_temporal<float, kLearn>(a, rect, use_id, grid, s);
        else launch_temporal<half_t, kLearn>(a, rect, use_id, grid, s);
    } else {
        if (t == SV_F32) launch_temporal<float, kBlend>(a, rect, use_id, grid, s);
        else launch_temporal<half_t, kBlend>(a, rect, use_id, grid, s);
    }
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
    const int rect = rect_mode(p);
    if (rect < 0) return SV_EINVAL;
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
                   p->alpha_m, p->gamma, p->tau_z, p->tau_n, p->tm_k, p->max_hist, tm ? 1 : 0,
                   io->g.dzdx, io->g.dzdy, albedo->r, albedo->g, albedo->b, (uint4 *)feat,
                   hist_out ? (float *)hist_out->r : nullptr,
                   hist_out ? (float *)hist_out->g : nullptr,
                   hist_out ? (float *)hist_out->b : nullptr, w->mu, w->inv_s};
    dim3 grid(xcd_grid(((d.w + kTX - 1) / kTX) * ((d.h + kTY - 1) / kTY)));
    hipStream_t s = as_stream(stream);
    if (t == SV_F32) launch_temporal<float, kFeat>(a, rect, use_id, grid, s);
    else launch_temporal<half_t, kFeat>(a, rect, use_id, grid, s);
    return hip_status(hipGetLastError());
}

static int clamp_or_clip(const sv_rgb *hist, const sv_rgb *cur, const sv_rgb *out, const void *z,
                         sv_dims d, sv_dtype t, float gamma, bool clip, sv_stream stream) {
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
    hipStream_t s = as_stream(stream);
    if (t == SV_F32) {
        if (clip) hipLaunchKernelGGL((clamp_k<float, kRectClip>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((clamp_k<float, kRectClamp>), grid, dim3(256), 0, s, a);
    } else {
        if (clip) hipLaunchKernelGGL((clamp_k<half_t, kRectClip>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((clamp_k<half_t, kRectClamp>), grid, dim3(256), 0, s, a);
    }
    return hip_status(hipGetLastError());
}

extern "C" int sv_clamp(const sv_rgb *hist, const sv_rgb *cur, const sv_rgb *out, const void *z,
                        sv_dims d, sv_dtype t, float gamma, sv_stream stream) {
    return clamp_or_clip(hist, cur, out, z, d, t, gamma, false, stream);
}

extern "C" int sv_clip(const sv_rgb *hist, const sv_rgb *cur, const sv_rgb *out, const void *z,
                       sv_dims d, sv_dtype t, float gamma, sv_stream stream) {
    return clamp_or_clip(hist, cur, out, z, d, t, gamma, true, stream);
}
