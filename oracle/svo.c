/*
 * FP64 CPU oracle of the SVGF-style denoiser described in "Hybrid-Rendering
 * Techniques in GPU" (Granja & Pereira, 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no source, header, table or helper with the HIP library.
 *
 * Every image is a contiguous row-major W x H array of doubles (pixel (x, y)
 * at index y*W + x); history lengths are int32.  Each step is one naive loop
 * per pixel, written in the order the method states it:
 *
 *   svo_tonemap      Reinhard tone map and its inverse (Section 3.4)
 *   svo_reproject    backward reprojection of the history (Section 2)
 *   svo_clamp        variance colour clamp of the history (Sections 2, 3.1)
 *   svo_clip         variance colour clipping of the history (Section 3.1)
 *   svo_blend        temporal accumulation of colour and moments (Section 2)
 *   svo_temporal     the four steps above in order (Section 3, step 4)
 *   svo_variance     per-pixel variance from the moments (Section 2)
 *   svo_atrous       one edge-avoiding a-trous level, 5x5 (Section 2, Fig. 1)
 *   svo_atrous_sep   one separable level, horizontal then vertical (Sec. 3.3)
 *   svo_quantize_half  binary16 round-to-nearest-even of stored colours
 *
 * The paper names these steps but prints no formula for them; the formulas
 * below are those of spatiotemporal variance-guided filtering and of the
 * edge-avoiding a-trous transform that Section 2 cites, and every choice the
 * paper leaves open is stated where it is made.
 *
 * Yes/no decisions taken from floating-point values (the depth and normal
 * tests of the reprojection) are evaluated in binary32 with a fixed
 * operation order, the precision of the device path; everything continuous
 * is FP64.  Build with -ffp-contract=off so that the compiler fuses nothing.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SVO_UNIT_WEIGHTS 1   /* a-trous: every edge-stopping weight is 1 */
#define SVO_INV_TONEMAP 2    /* a-trous: inverse tone map on the output */
#define SVO_HALF_OUT 4       /* round stored colour outputs to binary16 */

#define SVO_TM_LUMA 0        /* c / (1 + k L(c)) and its exact inverse */
#define SVO_TM_CHANNEL 1     /* c / (1 + k c) per channel and its inverse */
#define SVO_TM_PAPER 2       /* the listing's "inverse": c (1 + L(c)) w */

#define SVO_T_CLAMP 1        /* temporal: clamp the reprojected history */
#define SVO_T_USE_ID 2       /* temporal: object ids must match */
#define SVO_T_TONEMAP_IN 4   /* temporal: tone map the current colour first */
#define SVO_T_CLIP 8         /* temporal: clip the reprojected history instead */

/* Luminance with Rec. 709 weights (the listing's luma() is undefined). */
static double luma(double r, double g, double b)
{
    return 0.2126 * r + 0.7152 * g + 0.0722 * b;
}

/* A pixel without a surface (no hit) has a non-positive or non-finite
 * depth; it is passed through and never used as a neighbour. */
static int empty_px(double z)
{
    return !(z > 0.0) || !isfinite(z);
}

/* ---- binary16 rounding ------------------------------------------------ */

/* Round x to the nearest binary16 value, ties to even, straight from the
 * double (no intermediate binary32 rounding).  Overflow goes to infinity,
 * small values to subnormals or signed zero. */
static double round_half(double x)
{
    if (!isfinite(x) || x == 0.0)
        return x;
    double a = fabs(x);
    const double max_half = 65504.0;
    /* values at or beyond max + half an ulp (2^15 * 2^-11 / 2 = 16) overflow */
    if (a >= max_half + 16.0)
        return copysign(INFINITY, x);
    int e;
    frexp(a, &e);             /* a = m * 2^e with m in [0.5, 1) */
    int exp2 = e - 1;         /* a in [2^exp2, 2^(exp2+1)) */
    if (exp2 < -14)
        exp2 = -14;           /* subnormal range has the spacing of 2^-14 */
    double ulp = ldexp(1.0, exp2 - 10);
    double q = a / ulp;       /* exact: scaling by a power of two */
    double f = floor(q);
    double rem = q - f;
    if (rem > 0.5 || (rem == 0.5 && fmod(f, 2.0) != 0.0))
        f += 1.0;
    return copysign(f * ulp, x);
}

void svo_quantize_half(int64_t n, double *x)
{
    for (int64_t i = 0; i < n; ++i)
        x[i] = round_half(x[i]);
}

static void store_colour(double *dst, double v, int flags)
{
    *dst = (flags & SVO_HALF_OUT) ? round_half(v) : v;
}

/* ---- Section 3.4: Reinhard tone map ----------------------------------- */

/* Forward: the listing divides the radiance by 1 + luma * lumaMultiplier.
 * Inverse (mode LUMA): the exact inverse c' / (1 - k L(c')), because
 * L(c / (1 + k L(c))) = L(c) / (1 + k L(c)); the denominator is floored at
 * 2^-20.  Mode PAPER reproduces the listing's own "removal", which is not
 * an inverse: c' (1 + L(c')) w. */
void svo_tonemap(int64_t n, const double *r, const double *g, const double *b,
                 double *ro, double *go, double *bo, int inverse, int mode,
                 double k, double weight)
{
    for (int64_t i = 0; i < n; ++i) {
        double cr = r[i], cg = g[i], cb = b[i];
        double L = luma(cr, cg, cb);
        if (mode == SVO_TM_CHANNEL) {
            if (!inverse) {
                ro[i] = cr / (1.0 + k * cr);
                go[i] = cg / (1.0 + k * cg);
                bo[i] = cb / (1.0 + k * cb);
            } else {
                ro[i] = cr / fmax(1.0 - k * cr, 0x1p-20);
                go[i] = cg / fmax(1.0 - k * cg, 0x1p-20);
                bo[i] = cb / fmax(1.0 - k * cb, 0x1p-20);
            }
        } else if (!inverse) {
            double s = 1.0 / (1.0 + k * L);
            ro[i] = cr * s;
            go[i] = cg * s;
            bo[i] = cb * s;
        } else if (mode == SVO_TM_PAPER) {
            double s = (1.0 + L) * weight;
            ro[i] = cr * s;
            go[i] = cg * s;
            bo[i] = cb * s;
        } else {
            double s = 1.0 / fmax(1.0 - k * L, 0x1p-20);
            ro[i] = cr * s;
            go[i] = cg * s;
            bo[i] = cb * s;
        }
    }
}

/* ---- Section 2: backward reprojection ---------------------------------- */

/* binary32 decisions with a fixed operation order */
static int depth_consistent(float z_prev, float z_cur, float tau_z)
{
    float d = fabsf(z_prev - z_cur);
    float lim = tau_z * z_cur;
    return d <= lim;
}

static int normal_consistent(float ax, float ay, float az, float bx, float by,
                             float bz, float tau_n)
{
    float d = ax * bx;
    d = fmaf(ay, by, d);
    d = fmaf(az, bz, d);
    return d >= tau_n;
}

/* Pixel p = (x, y) was seen at q = p + mv(p) in the previous frame.  The
 * history is read there by bilinear interpolation over the four pixels
 * around q: x0 = x + floor(mv_x), fx = mv_x - floor(mv_x) (likewise y).  A
 * tap is usable when it lies in the image, holds history (length >= 1), its
 * previous depth and normal agree with p's current ones (and its object id,
 * if ids are used).  The usable taps' bilinear weights are renormalised; if
 * none with a positive weight is usable the history is discarded.  The
 * reprojected history length is the largest length among usable taps with
 * a positive weight. */
void svo_reproject(int W, int H, const double *z, const double *nx,
                   const double *ny, const double *nz, const uint8_t *id,
                   const double *mvx, const double *mvy, const double *pz,
                   const double *pnx, const double *pny, const double *pnz,
                   const uint8_t *pid, const double *hr, const double *hg,
                   const double *hb, const double *hm1, const double *hm2,
                   const int32_t *hn, double tau_z, double tau_n, int use_id,
                   double *or_, double *og, double *ob, double *om1,
                   double *om2, int32_t *on, int32_t *ovalid)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            or_[p] = og[p] = ob[p] = om1[p] = om2[p] = 0.0;
            on[p] = 0;
            ovalid[p] = 0;
            if (empty_px(z[p]))
                continue;
            /* motion that is not finite or beyond 2^20 pixels: no history */
            if (!(fabs(mvx[p]) < 1048576.0) || !(fabs(mvy[p]) < 1048576.0))
                continue;
            double fx0 = floor(mvx[p]), fy0 = floor(mvy[p]);
            double fx = mvx[p] - fx0, fy = mvy[p] - fy0;
            long x0 = x + (long)fx0, y0 = y + (long)fy0;
            double sw = 0.0, ar = 0.0, ag = 0.0, ab = 0.0, a1 = 0.0, a2 = 0.0;
            int nmax = 0, any = 0;
            for (int t = 0; t < 4; ++t) {
                long tx = x0 + (t & 1), ty = y0 + (t >> 1);
                double bw = ((t & 1) ? fx : 1.0 - fx) * ((t >> 1) ? fy : 1.0 - fy);
                if (!(bw > 0.0))
                    continue;
                if (tx < 0 || tx >= W || ty < 0 || ty >= H)
                    continue;
                int64_t q = (int64_t)ty * W + tx;
                if (hn[q] < 1)
                    continue;
                if (!depth_consistent((float)pz[q], (float)z[p], (float)tau_z))
                    continue;
                if (!normal_consistent((float)pnx[q], (float)pny[q], (float)pnz[q],
                                       (float)nx[p], (float)ny[p], (float)nz[p],
                                       (float)tau_n))
                    continue;
                if (use_id && id && pid && id[p] != pid[q])
                    continue;
                any = 1;
                sw += bw;
                ar += bw * hr[q];
                ag += bw * hg[q];
                ab += bw * hb[q];
                a1 += bw * hm1[q];
                a2 += bw * hm2[q];
                if (hn[q] > nmax)
                    nmax = hn[q];
            }
            if (!any)
                continue;
            or_[p] = ar / sw;
            og[p] = ag / sw;
            ob[p] = ab / sw;
            om1[p] = a1 / sw;
            om2[p] = a2 / sw;
            on[p] = nmax;
            ovalid[p] = 1;
        }
    }
}

/* ---- Sections 2 and 3.1: variance colour clamping ---------------------- */

/* Mean mu and population standard deviation sigma of the current colour
 * over the 3x3 neighbourhood of p (pixels in the image and not empty), per
 * channel, by the two-pass formula; the history colour is clamped to
 * [mu - gamma sigma, mu + gamma sigma].  gamma <= 0 copies the history.
 * `z` may be NULL (no empty pixels). */
void svo_clamp(int W, int H, const double *hr, const double *hg,
               const double *hb, const double *cr, const double *cg,
               const double *cb, const double *z, double gamma, double *or_,
               double *og, double *ob)
{
    const double *h[3] = {hr, hg, hb};
    const double *c[3] = {cr, cg, cb};
    double *o[3] = {or_, og, ob};
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            for (int ch = 0; ch < 3; ++ch) {
                double v = h[ch][p];
                if (gamma > 0.0 && !(z && empty_px(z[p]))) {
                    double sum = 0.0;
                    int cnt = 0;
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int qx = x + dx, qy = y + dy;
                            if (qx < 0 || qx >= W || qy < 0 || qy >= H)
                                continue;
                            int64_t q = (int64_t)qy * W + qx;
                            if (z && empty_px(z[q]))
                                continue;
                            sum += c[ch][q];
                            ++cnt;
                        }
                    double mu = sum / cnt;
                    double ss = 0.0;
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int qx = x + dx, qy = y + dy;
                            if (qx < 0 || qx >= W || qy < 0 || qy >= H)
                                continue;
                            int64_t q = (int64_t)qy * W + qx;
                            if (z && empty_px(z[q]))
                                continue;
                            double d = c[ch][q] - mu;
                            ss += d * d;
                        }
                    double sigma = sqrt(ss / cnt);
                    double lo = mu - gamma * sigma, hi = mu + gamma * sigma;
                    v = fmin(fmax(v, lo), hi);
                }
                o[ch][p] = v;
            }
        }
    }
}

/* Variance colour clipping, the alternative Section 3.1 tested beside the
 * clamp.  The box is the same (centre mu, half-widths gamma sigma per
 * channel, from the 3x3 neighbourhood of the current colour), but a history
 * colour outside it is moved toward mu along the segment from mu, onto the
 * box's surface, rather than channel by channel: with d = h - mu and
 * t = min(1, min over channels with |d_c| > gamma sigma_c of
 * gamma sigma_c / |d_c|), the result is mu + t d.  The hue of the history
 * is kept.  A channel with zero spread and a nonzero deviation gives t = 0,
 * i.e. mu.  A history inside the box is kept as it is; gamma <= 0 copies
 * the history. */
void svo_clip(int W, int H, const double *hr, const double *hg,
              const double *hb, const double *cr, const double *cg,
              const double *cb, const double *z, double gamma, double *or_,
              double *og, double *ob)
{
    const double *h[3] = {hr, hg, hb};
    const double *c[3] = {cr, cg, cb};
    double *o[3] = {or_, og, ob};
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            if (!(gamma > 0.0) || (z && empty_px(z[p]))) {
                for (int ch = 0; ch < 3; ++ch)
                    o[ch][p] = h[ch][p];
                continue;
            }
            double mu[3], half[3];
            for (int ch = 0; ch < 3; ++ch) {
                double sum = 0.0;
                int cnt = 0;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int qx = x + dx, qy = y + dy;
                        if (qx < 0 || qx >= W || qy < 0 || qy >= H)
                            continue;
                        int64_t q = (int64_t)qy * W + qx;
                        if (z && empty_px(z[q]))
                            continue;
                        sum += c[ch][q];
                        ++cnt;
                    }
                mu[ch] = sum / cnt;
                double ss = 0.0;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int qx = x + dx, qy = y + dy;
                        if (qx < 0 || qx >= W || qy < 0 || qy >= H)
                            continue;
                        int64_t q = (int64_t)qy * W + qx;
                        if (z && empty_px(z[q]))
                            continue;
                        double d = c[ch][q] - mu[ch];
                        ss += d * d;
                    }
                half[ch] = gamma * sqrt(ss / cnt);
            }
            double t = 1.0;
            for (int ch = 0; ch < 3; ++ch) {
                double d = fabs(h[ch][p] - mu[ch]);
                if (d > half[ch])
                    t = fmin(t, half[ch] / d);
            }
            for (int ch = 0; ch < 3; ++ch)
                o[ch][p] = t < 1.0 ? mu[ch] + t * (h[ch][p] - mu[ch]) : h[ch][p];
        }
    }
}

/* ---- Section 2: temporal accumulation ---------------------------------- */

/* Exponential moving average of colour and of the first two luminance
 * moments.  The blend weight is max(alpha, 1/n) with n the new history
 * length, so the first frames of a history are a plain running mean.  A
 * discarded history restarts from the current sample (n = 1).  An empty
 * pixel passes its colour through with zero moments and n = 0.
 * `alpha_map` (may be NULL) gives a per-pixel colour alpha instead of
 * `alpha`. */
void svo_blend(int64_t npx, const double *cr, const double *cg,
               const double *cb, const double *z, const double *hr,
               const double *hg, const double *hb, const double *hm1,
               const double *hm2, const int32_t *hn, const int32_t *valid,
               double alpha, double alpha_m, const double *alpha_map,
               int max_hist, int flags, double *or_, double *og, double *ob,
               double *om1, double *om2, int32_t *on)
{
    for (int64_t p = 0; p < npx; ++p) {
        double L = luma(cr[p], cg[p], cb[p]);
        if (empty_px(z[p])) {
            store_colour(&or_[p], cr[p], flags);
            store_colour(&og[p], cg[p], flags);
            store_colour(&ob[p], cb[p], flags);
            om1[p] = 0.0;
            om2[p] = 0.0;
            on[p] = 0;
            continue;
        }
        if (!valid[p]) {
            store_colour(&or_[p], cr[p], flags);
            store_colour(&og[p], cg[p], flags);
            store_colour(&ob[p], cb[p], flags);
            om1[p] = L;
            om2[p] = L * L;
            on[p] = 1;
            continue;
        }
        int n = hn[p] + 1;
        if (n > max_hist)
            n = max_hist;
        double a_c = alpha_map ? alpha_map[p] : alpha;
        a_c = fmax(a_c, 1.0 / n);
        double a_m = fmax(alpha_m, 1.0 / n);
        store_colour(&or_[p], (1.0 - a_c) * hr[p] + a_c * cr[p], flags);
        store_colour(&og[p], (1.0 - a_c) * hg[p] + a_c * cg[p], flags);
        store_colour(&ob[p], (1.0 - a_c) * hb[p] + a_c * cb[p], flags);
        om1[p] = (1.0 - a_m) * hm1[p] + a_m * L;
        om2[p] = (1.0 - a_m) * hm2[p] + a_m * L * L;
        on[p] = n;
    }
}

/* The whole temporal filter of Section 3 step 4, in order: (tone map the
 * current colour), reproject the history, (clamp or clip it), blend.  `cur` is the
 * raw current colour; scratch is allocated here. */
int svo_temporal(int W, int H, const double *cr, const double *cg,
                 const double *cb, const double *z, const double *nx,
                 const double *ny, const double *nz, const uint8_t *id,
                 const double *mvx, const double *mvy, const double *pz,
                 const double *pnx, const double *pny, const double *pnz,
                 const uint8_t *pid, const double *hr, const double *hg,
                 const double *hb, const double *hm1, const double *hm2,
                 const int32_t *hn, double alpha, double alpha_m, double gamma,
                 double tau_z, double tau_n, double tm_k, int max_hist,
                 int flags, int out_flags, const double *alpha_map,
                 double *or_, double *og, double *ob, double *om1,
                 double *om2, int32_t *on)
{
    int64_t n = (int64_t)W * H;
    double *buf = (double *)malloc(sizeof(double) * n * 11);
    int32_t *ibuf = (int32_t *)malloc(sizeof(int32_t) * n * 2);
    if (!buf || !ibuf) {
        free(buf);
        free(ibuf);
        return -1;
    }
    double *tr = buf, *tg = buf + n, *tb = buf + 2 * n;
    double *rr = buf + 3 * n, *rg = buf + 4 * n, *rb = buf + 5 * n;
    double *r1 = buf + 6 * n, *r2 = buf + 7 * n;
    double *kr = buf + 8 * n, *kg = buf + 9 * n, *kb = buf + 10 * n;
    int32_t *rn = ibuf, *rv = ibuf + n;
    if (flags & SVO_T_TONEMAP_IN) {
        svo_tonemap(n, cr, cg, cb, tr, tg, tb, 0, SVO_TM_LUMA, tm_k, 1.0);
    } else {
        memcpy(tr, cr, sizeof(double) * n);
        memcpy(tg, cg, sizeof(double) * n);
        memcpy(tb, cb, sizeof(double) * n);
    }
    svo_reproject(W, H, z, nx, ny, nz, id, mvx, mvy, pz, pnx, pny, pnz, pid,
                  hr, hg, hb, hm1, hm2, hn, tau_z, tau_n,
                  (flags & SVO_T_USE_ID) != 0, rr, rg, rb, r1, r2, rn, rv);
    if ((flags & SVO_T_CLIP) && gamma > 0.0) {
        svo_clip(W, H, rr, rg, rb, tr, tg, tb, z, gamma, kr, kg, kb);
    } else if ((flags & SVO_T_CLAMP) && gamma > 0.0) {
        svo_clamp(W, H, rr, rg, rb, tr, tg, tb, z, gamma, kr, kg, kb);
    } else {
        memcpy(kr, rr, sizeof(double) * n);
        memcpy(kg, rg, sizeof(double) * n);
        memcpy(kb, rb, sizeof(double) * n);
    }
    svo_blend(n, tr, tg, tb, z, kr, kg, kb, r1, r2, rn, rv, alpha, alpha_m,
              alpha_map, max_hist, out_flags, or_, og, ob, om1, om2, on);
    free(buf);
    free(ibuf);
    return 0;
}

/* ---- edge-stopping functions (Section 2) ------------------------------ */

/* Depth: the depth difference relative to the difference that p's screen
 * depth gradient predicts over the offset (dx, dy). */
static double w_depth(double zp, double zq, double gx, double gy, double dx,
                      double dy, double sigma_z, double eps_z)
{
    return exp(-fabs(zp - zq) / (sigma_z * fabs(gx * dx + gy * dy) + eps_z));
}

/* Normal: a power of the clamped cosine between the two unit normals,
 * the cosine taken as 1 - |n(p) - n(q)|^2 / 2 (the same value for unit
 * vectors; for G-buffer normals rounded to binary32 or binary16 it stays a
 * function of the angle alone). */
static double w_normal(double ax, double ay, double az, double bx, double by,
                       double bz, double sigma_n)
{
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    double d = 1.0 - 0.5 * (dx * dx + dy * dy + dz * dz);
    return pow(d > 0.0 ? d : 0.0, sigma_n);
}

/* Luminance: the luminance difference relative to the standard deviation
 * that p's (prefiltered) variance predicts: low variance, little mixing. */
static double w_luma(double lp, double lq, double sigma_l, double kappa,
                     double g, double eps_l)
{
    return exp(-fabs(lp - lq) / (sigma_l * kappa * sqrt(g) + eps_l));
}

/* ---- Section 2: variance estimate -------------------------------------- */

/* With a history of at least min_hist frames the variance is the temporal
 * one, m2 - m1^2 (floored at zero).  A shorter history has too few samples,
 * so the moments are averaged over a (2 radius + 1)^2 window with depth and
 * normal weights (the centre weighs 1) and the variance of the mixture is
 * taken in split form: weighted mean of (m2 - m1^2) plus the weighted
 * spread of m1 around its weighted mean, which equals mean(m2) - mean(m1)^2
 * without its cancellation.  Empty pixels get zero. */
void svo_variance(int W, int H, const double *m1, const double *m2,
                  const int32_t *hn, const double *z, const double *dzdx,
                  const double *dzdy, const double *nx, const double *ny,
                  const double *nz, double sigma_z, double sigma_n,
                  double eps_z, int min_hist, int radius, double *var)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            if (empty_px(z[p]) || hn[p] < 1) {
                var[p] = 0.0;
                continue;
            }
            if (hn[p] >= min_hist) {
                double v = m2[p] - m1[p] * m1[p];
                var[p] = v > 0.0 ? v : 0.0;
                continue;
            }
            double sw = 0.0, s1 = 0.0;
            for (int dy = -radius; dy <= radius; ++dy)
                for (int dx = -radius; dx <= radius; ++dx) {
                    int qx = x + dx, qy = y + dy;
                    if (qx < 0 || qx >= W || qy < 0 || qy >= H)
                        continue;
                    int64_t q = (int64_t)qy * W + qx;
                    if (empty_px(z[q]))
                        continue;
                    double w = 1.0;
                    if (q != p)
                        w = w_depth(z[p], z[q], dzdx[p], dzdy[p], dx, dy, sigma_z, eps_z)
                            * w_normal(nx[p], ny[p], nz[p], nx[q], ny[q], nz[q], sigma_n);
                    sw += w;
                    s1 += w * m1[q];
                }
            double mean1 = s1 / sw;
            double within = 0.0, spread = 0.0;
            for (int dy = -radius; dy <= radius; ++dy)
                for (int dx = -radius; dx <= radius; ++dx) {
                    int qx = x + dx, qy = y + dy;
                    if (qx < 0 || qx >= W || qy < 0 || qy >= H)
                        continue;
                    int64_t q = (int64_t)qy * W + qx;
                    if (empty_px(z[q]))
                        continue;
                    double w = 1.0;
                    if (q != p)
                        w = w_depth(z[p], z[q], dzdx[p], dzdy[p], dx, dy, sigma_z, eps_z)
                            * w_normal(nx[p], ny[p], nz[p], nx[q], ny[q], nz[q], sigma_n);
                    within += w * (m2[q] - m1[q] * m1[q]);
                    double d = m1[q] - mean1;
                    spread += w * d * d;
                }
            double v = within / sw + spread / sw;
            var[p] = v > 0.0 ? v : 0.0;
        }
    }
}

/* ---- Section 2, Fig. 1: edge-avoiding a-trous level -------------------- */

/* B3-spline taps of the a-trous kernel and the 3x3 Gaussian that prefilters
 * the variance before it scales the luminance weight. */
static const double B3[5] = {1.0 / 16, 1.0 / 4, 3.0 / 8, 1.0 / 4, 1.0 / 16};
static const double G3[3] = {0.25, 0.5, 0.25};

static double prefiltered_variance(int W, int H, const double *var,
                                   const double *z, int x, int y)
{
    double s = 0.0, sw = 0.0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            int qx = x + dx, qy = y + dy;
            if (qx < 0 || qx >= W || qy < 0 || qy >= H)
                continue;
            int64_t q = (int64_t)qy * W + qx;
            if (empty_px(z[q]))
                continue;
            double k = G3[dx + 1] * G3[dy + 1];
            s += k * var[q];
            sw += k;
        }
    return s / sw;
}

static void inverse_tonemap_px(double *r, double *g, double *b, double k)
{
    double L = luma(*r, *g, *b);
    double s = 1.0 / fmax(1.0 - k * L, 0x1p-20);
    *r *= s;
    *g *= s;
    *b *= s;
}

/* One level with hole spacing `step`: taps q = p + step (a, b) for a, b in
 * -2..2 that lie in the image and are not empty.  Weight H(a, b) w(p, q)
 * with H the outer product of the B3 taps and w the product of the depth,
 * normal and luminance weights (w = 1 at q = p).  The colour is the
 * normalised weighted mean; the variance is propagated with the squared
 * weights:  var' = sum (H w)^2 var(q) / (sum H w)^2.  `kappa` (may be NULL)
 * scales sigma_l per pixel.  `var_out` may be NULL (last level). */
void svo_atrous(int W, int H, const double *cr, const double *cg,
                const double *cb, const double *var, const double *z,
                const double *dzdx, const double *dzdy, const double *nx,
                const double *ny, const double *nz, const double *kappa,
                int step, double sigma_z, double sigma_n, double sigma_l,
                double eps_z, double eps_l, double tm_k, int flags,
                double *or_, double *og, double *ob, double *var_out)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            double r, g, b, v;
            if (empty_px(z[p])) {
                r = cr[p];
                g = cg[p];
                b = cb[p];
                v = 0.0;
            } else {
                double lp = luma(cr[p], cg[p], cb[p]);
                double gv = prefiltered_variance(W, H, var, z, x, y);
                double kp = kappa ? kappa[p] : 1.0;
                double sw = 0.0, sr = 0.0, sg = 0.0, sb = 0.0, sv = 0.0;
                for (int bj = -2; bj <= 2; ++bj)
                    for (int ai = -2; ai <= 2; ++ai) {
                        int qx = x + step * ai, qy = y + step * bj;
                        if (qx < 0 || qx >= W || qy < 0 || qy >= H)
                            continue;
                        int64_t q = (int64_t)qy * W + qx;
                        if (empty_px(z[q]))
                            continue;
                        double w = 1.0;
                        if (q != p && !(flags & SVO_UNIT_WEIGHTS)) {
                            double lq = luma(cr[q], cg[q], cb[q]);
                            w = w_depth(z[p], z[q], dzdx[p], dzdy[p],
                                        (double)step * ai, (double)step * bj,
                                        sigma_z, eps_z)
                                * w_normal(nx[p], ny[p], nz[p], nx[q], ny[q], nz[q], sigma_n)
                                * w_luma(lp, lq, sigma_l, kp, gv, eps_l);
                        }
                        double hw = B3[ai + 2] * B3[bj + 2] * w;
                        sw += hw;
                        sr += hw * cr[q];
                        sg += hw * cg[q];
                        sb += hw * cb[q];
                        sv += hw * hw * var[q];
                    }
                r = sr / sw;
                g = sg / sw;
                b = sb / sw;
                v = sv / (sw * sw);
            }
            if (flags & SVO_INV_TONEMAP)
                inverse_tonemap_px(&r, &g, &b, tm_k);
            store_colour(&or_[p], r, flags);
            store_colour(&og[p], g, flags);
            store_colour(&ob[p], b, flags);
            if (var_out)
                var_out[p] = v;
        }
    }
}

/* ---- Section 3.3: separable level --------------------------------------- */

/* The 5x5 level split into a horizontal pass and a vertical pass, 5 taps
 * each (10 visits per pixel instead of 25).  Both passes use the variance
 * prefiltered from the level's input.  The horizontal pass filters colour
 * only (its result is stored like any colour); the vertical pass filters
 * that result and is the only one that updates the variance:
 * var' = sum (h w)^2 var_in(q) / (sum h w)^2 over the vertical taps.
 * `sh_r/g/b` receive the horizontal result (W*H each). */
void svo_atrous_sep(int W, int H, const double *cr, const double *cg,
                    const double *cb, const double *var, const double *z,
                    const double *dzdx, const double *dzdy, const double *nx,
                    const double *ny, const double *nz, const double *kappa,
                    int step, double sigma_z, double sigma_n, double sigma_l,
                    double eps_z, double eps_l, double tm_k, int flags,
                    double *sh_r, double *sh_g, double *sh_b, double *or_,
                    double *og, double *ob, double *var_out)
{
    int64_t n = (int64_t)W * H;
    double *gbuf = (double *)malloc(sizeof(double) * n);
    if (!gbuf)
        return;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            gbuf[p] = empty_px(z[p]) ? 0.0 : prefiltered_variance(W, H, var, z, x, y);
        }
    /* horizontal pass */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            double r = cr[p], g = cg[p], b = cb[p];
            if (!empty_px(z[p])) {
                double lp = luma(cr[p], cg[p], cb[p]);
                double kp = kappa ? kappa[p] : 1.0;
                double sw = 0.0, sr = 0.0, sg = 0.0, sb = 0.0;
                for (int ai = -2; ai <= 2; ++ai) {
                    int qx = x + step * ai;
                    if (qx < 0 || qx >= W)
                        continue;
                    int64_t q = (int64_t)y * W + qx;
                    if (empty_px(z[q]))
                        continue;
                    double w = 1.0;
                    if (q != p && !(flags & SVO_UNIT_WEIGHTS)) {
                        double lq = luma(cr[q], cg[q], cb[q]);
                        w = w_depth(z[p], z[q], dzdx[p], dzdy[p], (double)step * ai, 0.0,
                                    sigma_z, eps_z)
                            * w_normal(nx[p], ny[p], nz[p], nx[q], ny[q], nz[q], sigma_n)
                            * w_luma(lp, lq, sigma_l, kp, gbuf[p], eps_l);
                    }
                    double hw = B3[ai + 2] * w;
                    sw += hw;
                    sr += hw * cr[q];
                    sg += hw * cg[q];
                    sb += hw * cb[q];
                }
                r = sr / sw;
                g = sg / sw;
                b = sb / sw;
            }
            store_colour(&sh_r[p], r, flags & SVO_HALF_OUT);
            store_colour(&sh_g[p], g, flags & SVO_HALF_OUT);
            store_colour(&sh_b[p], b, flags & SVO_HALF_OUT);
        }
    }
    /* vertical pass */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            double r = sh_r[p], g = sh_g[p], b = sh_b[p], v = 0.0;
            if (!empty_px(z[p])) {
                double lp = luma(sh_r[p], sh_g[p], sh_b[p]);
                double kp = kappa ? kappa[p] : 1.0;
                double sw = 0.0, sr = 0.0, sg = 0.0, sb = 0.0, sv = 0.0;
                for (int bj = -2; bj <= 2; ++bj) {
                    int qy = y + step * bj;
                    if (qy < 0 || qy >= H)
                        continue;
                    int64_t q = (int64_t)qy * W + x;
                    if (empty_px(z[q]))
                        continue;
                    double w = 1.0;
                    if (q != p && !(flags & SVO_UNIT_WEIGHTS)) {
                        double lq = luma(sh_r[q], sh_g[q], sh_b[q]);
                        w = w_depth(z[p], z[q], dzdx[p], dzdy[p], 0.0, (double)step * bj,
                                    sigma_z, eps_z)
                            * w_normal(nx[p], ny[p], nz[p], nx[q], ny[q], nz[q], sigma_n)
                            * w_luma(lp, lq, sigma_l, kp, gbuf[p], eps_l);
                    }
                    double hw = B3[bj + 2] * w;
                    sw += hw;
                    sr += hw * sh_r[q];
                    sg += hw * sh_g[q];
                    sb += hw * sh_b[q];
                    sv += hw * hw * var[q];
                }
                r = sr / sw;
                g = sg / sw;
                b = sb / sw;
                v = sv / (sw * sw);
            }
            if (flags & SVO_INV_TONEMAP)
                inverse_tonemap_px(&r, &g, &b, tm_k);
            store_colour(&or_[p], r, flags);
            store_colour(&og[p], g, flags);
            store_colour(&ob[p], b, flags);
            if (var_out)
                var_out[p] = v;
        }
    }
    free(gbuf);
}

int svo_version(void)
{
    return 1;
}

/* Host threads of the parallel loops (timing only: every result is the
 * same at any count, each pixel being computed by one thread alone). */
void svo_set_threads(int n)
{
    omp_set_num_threads(n > 0 ? n : 1);
}

int svo_threads(void)
{
    return omp_get_max_threads();
}
