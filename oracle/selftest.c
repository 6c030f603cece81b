/* Memory- and UB-safety self-test of the FP64 oracle (svo.c).
 *
 * TEST INFRASTRUCTURE ONLY.  Built together with svo.c under AddressSanitizer
 * and UndefinedBehaviorSanitizer (host code only, gcc), it calls every
 * exported svo_* routine on degenerate and ragged image sizes (1x1, one row,
 * one column, sizes smaller than the a-trous step), with the inputs the
 * filter has to survive: empty pixels (zero, negative and non-finite depth),
 * motion vectors off the image, non-finite and huge, history lengths of zero,
 * every flag combination and two thread counts.  Any
 * out-of-bounds access, leak or undefined operation aborts the run with the
 * sanitizer's report; the driver itself also checks that every output plane
 * was written (a canary value must not survive) and that, for finite inputs,
 * the outputs are finite.
 *
 * Exit status 0 and the last line "selftest ok <cases>" mean every case ran
 * clean. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void svo_quantize_half(int64_t n, double *x);
void svo_tonemap(int64_t n, const double *r, const double *g, const double *b,
                 double *ro, double *go, double *bo, int inverse, int mode,
                 double k, double weight);
void svo_reproject(int W, int H, const double *z, const double *nx,
                   const double *ny, const double *nz, const uint8_t *id,
                   const double *mvx, const double *mvy, const double *pz,
                   const double *pnx, const double *pny, const double *pnz,
                   const uint8_t *pid, const double *hr, const double *hg,
                   const double *hb, const double *hm1, const double *hm2,
                   const int32_t *hn, double tau_z, double tau_n, int use_id,
                   double *or_, double *og, double *ob, double *om1,
                   double *om2, int32_t *on, int32_t *ovalid);
void svo_clamp(int W, int H, const double *hr, const double *hg,
               const double *hb, const double *cr, const double *cg,
               const double *cb, const double *z, double gamma, double *or_,
               double *og, double *ob);
void svo_clip(int W, int H, const double *hr, const double *hg,
              const double *hb, const double *cr, const double *cg,
              const double *cb, const double *z, double gamma, double *or_,
              double *og, double *ob);
void svo_blend(int64_t npx, const double *cr, const double *cg,
               const double *cb, const double *z, const double *hr,
               const double *hg, const double *hb, const double *hm1,
               const double *hm2, const int32_t *hn, const int32_t *valid,
               double alpha, double alpha_m, const double *alpha_map,
               int max_hist, int flags, double *or_, double *og, double *ob,
               double *om1, double *om2, int32_t *on);
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
                 double *om2, int32_t *on);
void svo_variance(int W, int H, const double *m1, const double *m2,
                  const int32_t *hn, const double *z, const double *dzdx,
                  const double *dzdy, const double *nx, const double *ny,
                  const double *nz, double sigma_z, double sigma_n,
                  double eps_z, int min_hist, int radius, double *var);
void svo_atrous(int W, int H, const double *cr, const double *cg,
                const double *cb, const double *var, const double *z,
                const double *dzdx, const double *dzdy, const double *nx,
                const double *ny, const double *nz, const double *kappa,
                int step, double sigma_z, double sigma_n, double sigma_l,
                double eps_z, double eps_l, double tm_k, int flags,
                double *or_, double *og, double *ob, double *var_out);
void svo_atrous_sep(int W, int H, const double *cr, const double *cg,
                    const double *cb, const double *var, const double *z,
                    const double *dzdx, const double *dzdy, const double *nx,
                    const double *ny, const double *nz, const double *kappa,
                    int step, double sigma_z, double sigma_n, double sigma_l,
                    double eps_z, double eps_l, double tm_k, int flags,
                    double *sh_r, double *sh_g, double *sh_b, double *or_,
                    double *og, double *ob, double *var_out);
int svo_version(void);
void svo_set_threads(int n);
int svo_threads(void);

/* Flag values of svo.c's interface. */
enum { UNIT_WEIGHTS = 1, INV_TONEMAP = 2, HALF_OUT = 4 };
enum { T_CLAMP = 1, T_USE_ID = 2, T_TONEMAP_IN = 4, T_CLIP = 8 };

static const double CANARY = -1234567.25;
static long g_cases = 0;
static int g_fail = 0;

/* xorshift64*: a seeded stream of doubles in [0, 1). */
static uint64_t g_rng = 0x9e3779b97f4a7c15ull;
static double urand(void)
{
    g_rng ^= g_rng >> 12;
    g_rng ^= g_rng << 25;
    g_rng ^= g_rng >> 27;
    return (double)((g_rng * 2685821657736338717ull) >> 11) * 0x1.0p-53;
}

/* Planes are allocated to their exact size so that ASan sees any access
 * one element past the end. */
static double *plane(int64_t n)
{
    double *p = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    for (int64_t i = 0; i < n; ++i)
        p[i] = CANARY;
    return p;
}

static int32_t *iplane(int64_t n)
{
    int32_t *p = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    for (int64_t i = 0; i < n; ++i)
        p[i] = -77;
    return p;
}

/* Refill output planes with the canary so that each call's check sees only
 * what that call wrote. */
static void canary(int64_t n, double *a, double *b, double *c)
{
    double *p[3] = {a, b, c};
    for (int k = 0; k < 3; ++k)
        if (p[k])
            for (int64_t i = 0; i < n; ++i)
                p[k][i] = CANARY;
}

static double *uniform(int64_t n, double lo, double hi)
{
    double *p = plane(n);
    for (int64_t i = 0; i < n; ++i)
        p[i] = lo + (hi - lo) * urand();
    return p;
}

static void check_written(const char *what, int W, int H, const double *p,
                          int want_finite)
{
    int64_t n = (int64_t)W * H;
    for (int64_t i = 0; i < n; ++i) {
        if (p[i] == CANARY || (want_finite && !isfinite(p[i]))) {
            fprintf(stderr, "FAIL %s %dx%d at %lld: %g\n", what, W, H,
                    (long long)i, p[i]);
            g_fail = 1;
            return;
        }
    }
}

static void check_iwritten(const char *what, int W, int H, const int32_t *p,
                           int lo, int hi)
{
    int64_t n = (int64_t)W * H;
    for (int64_t i = 0; i < n; ++i) {
        if (p[i] < lo || p[i] > hi) {
            fprintf(stderr, "FAIL %s %dx%d at %lld: %d\n", what, W, H,
                    (long long)i, p[i]);
            g_fail = 1;
            return;
        }
    }
}

/* One frame's G-buffer and history on a W x H image.  `hostile` plants
 * empty pixels of every kind, motion off the image, non-finite and beyond
 * the oracle's 2^20-pixel cut-off, and zero-length histories. */
typedef struct {
    int W, H;
    double *cr, *cg, *cb, *z, *nx, *ny, *nz, *dzdx, *dzdy, *mvx, *mvy;
    double *pz, *pnx, *pny, *pnz, *hr, *hg, *hb, *hm1, *hm2, *amap, *kappa;
    uint8_t *id, *pid;
    int32_t *hn;
} frame_t;

static void frame_new(frame_t *f, int W, int H, int hostile)
{
    int64_t n = (int64_t)W * H;
    f->W = W;
    f->H = H;
    f->cr = uniform(n, 0.0, 4.0);
    f->cg = uniform(n, 0.0, 4.0);
    f->cb = uniform(n, 0.0, 4.0);
    f->z = uniform(n, 0.5, 2.0);
    f->dzdx = uniform(n, -0.05, 0.05);
    f->dzdy = uniform(n, -0.05, 0.05);
    f->nx = plane(n);
    f->ny = plane(n);
    f->nz = plane(n);
    f->pnx = plane(n);
    f->pny = plane(n);
    f->pnz = plane(n);
    for (int64_t i = 0; i < n; ++i) {
        double a = 6.283185307179586 * urand(), c = 0.2 + 0.8 * urand();
        double s = sqrt(1.0 - c * c);
        f->nx[i] = s * cos(a);
        f->ny[i] = s * sin(a);
        f->nz[i] = c;
        f->pnx[i] = f->nx[i];
        f->pny[i] = f->ny[i];
        f->pnz[i] = f->nz[i];
    }
    f->mvx = uniform(n, -2.5, 2.5);
    f->mvy = uniform(n, -2.5, 2.5);
    f->pz = plane(n);
    for (int64_t i = 0; i < n; ++i)
        f->pz[i] = f->z[i] * (1.0 + 0.01 * (urand() - 0.5));
    f->hr = uniform(n, 0.0, 3.0);
    f->hg = uniform(n, 0.0, 3.0);
    f->hb = uniform(n, 0.0, 3.0);
    f->hm1 = uniform(n, 0.0, 2.0);
    f->hm2 = plane(n);
    for (int64_t i = 0; i < n; ++i)
        f->hm2[i] = f->hm1[i] * f->hm1[i] + urand();
    f->amap = uniform(n, 0.0, 1.0);
    f->kappa = uniform(n, 0.25, 8.0);
    f->hn = iplane(n);
    for (int64_t i = 0; i < n; ++i)
        f->hn[i] = (int32_t)(urand() * 40.0);
    f->id = malloc((size_t)(n > 0 ? n : 1));
    f->pid = malloc((size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        f->id[i] = (uint8_t)(urand() * 3.0);
        f->pid[i] = urand() < 0.8 ? f->id[i] : (uint8_t)(urand() * 3.0);
    }
    if (!hostile)
        return;
    static const double bad_z[] = {0.0, -1.0, NAN, INFINITY, -0.0};
    static const double bad_mv[] = {1e7, -1e7, NAN, INFINITY, 1048575.5,
                                    -1048576.0, 3.0 * 1048576.0};
    for (int64_t i = 0; i < n; ++i) {
        double u = urand();
        if (u < 0.15)
            f->z[i] = bad_z[(int)(urand() * 5.0)];
        else if (u < 0.25)
            f->pz[i] = bad_z[(int)(urand() * 5.0)];
        u = urand();
        if (u < 0.1) {
            f->mvx[i] = bad_mv[(int)(urand() * 7.0)];
            f->mvy[i] = bad_mv[(int)(urand() * 7.0)];
        } else if (u < 0.2) {
            f->mvx[i] = (urand() - 0.5) * 4.0 * (W + 2);
            f->mvy[i] = (urand() - 0.5) * 4.0 * (H + 2);
        } else if (u < 0.25) {
            f->mvx[i] = -(double)(i % W) - 0.5;   /* taps straddle x = -1 */
            f->mvy[i] = (double)(H - 1 - i / W) + 0.25; /* and y = H - 1 */
        }
        if (urand() < 0.2)
            f->hn[i] = 0;
    }
}

static void frame_free(frame_t *f)
{
    double *planes[] = {f->cr, f->cg, f->cb, f->z, f->nx, f->ny, f->nz,
                        f->dzdx, f->dzdy, f->mvx, f->mvy, f->pz, f->pnx,
                        f->pny, f->pnz, f->hr, f->hg, f->hb, f->hm1, f->hm2,
                        f->amap, f->kappa};
    for (size_t i = 0; i < sizeof planes / sizeof planes[0]; ++i)
        free(planes[i]);
    free(f->hn);
    free(f->id);
    free(f->pid);
}

static void case_half(void)
{
    double v[] = {0.0, -0.0, 1.0, 65504.0, 65519.99, 65520.0, -65520.0,
                  0x1p-24, 0x1p-25, 0x1.8p-25, 0x1p-26, 1e-300, -1e-300,
                  NAN, INFINITY, -INFINITY, 1e300, 2049.0, 2051.0, 0.1};
    int64_t n = (int64_t)(sizeof v / sizeof v[0]);
    double *x = plane(n);
    memcpy(x, v, sizeof v);
    svo_quantize_half(n, x);
    ++g_cases;
    if (x[5] != INFINITY || x[4] != 65504.0 || x[7] != 0x1p-24 ||
        x[8] != 0.0 || x[9] != 0x1p-24 || x[17] != 2048.0 || x[18] != 2052.0 ||
        !isnan(x[13])) {
        fprintf(stderr, "FAIL quantize_half specials\n");
        g_fail = 1;
    }
    free(x);
    svo_quantize_half(0, NULL);
}

static void case_frame(int W, int H, int hostile)
{
    frame_t f;
    frame_new(&f, W, H, hostile);
    int64_t n = (int64_t)W * H;
    double *o[13];
    for (int i = 0; i < 13; ++i)
        o[i] = plane(n);
    int32_t *on = iplane(n), *ov = iplane(n), *on2 = iplane(n);

    for (int mode = 0; mode < 3; ++mode)
        for (int inv = 0; inv < 2; ++inv) {
            canary(n, o[0], o[1], o[2]);
            svo_tonemap(n, f.cr, f.cg, f.cb, o[0], o[1], o[2], inv, mode, 1.5,
                        0.75);
            ++g_cases;
            check_written("tonemap", W, H, o[0], 1);
        }

    for (int use_id = 0; use_id < 2; ++use_id) {
        canary(n, o[0], o[1], o[2]);
        canary(n, o[3], o[4], NULL);
        svo_reproject(W, H, f.z, f.nx, f.ny, f.nz, f.id, f.mvx, f.mvy, f.pz,
                      f.pnx, f.pny, f.pnz, f.pid, f.hr, f.hg, f.hb, f.hm1,
                      f.hm2, f.hn, 0.05, 0.9, use_id, o[0], o[1], o[2], o[3],
                      o[4], on, ov);
        ++g_cases;
        check_written("reproject", W, H, o[0], 1);
        check_written("reproject m2", W, H, o[4], 1);
        check_iwritten("reproject n", W, H, on, 0, 40);
        check_iwritten("reproject valid", W, H, ov, 0, 1);
    }

    for (int clip = 0; clip < 2; ++clip)
        for (int withz = 0; withz < 2; ++withz)
            for (int gi = 0; gi < 3; ++gi) {
                const double gam[] = {0.0, 1.0, 3.5};
                canary(n, o[0], o[1], o[2]);
                (clip ? svo_clip : svo_clamp)(
                    W, H, f.hr, f.hg, f.hb, f.cr, f.cg, f.cb,
                    withz ? f.z : NULL, gam[gi], o[0], o[1], o[2]);
                ++g_cases;
                check_written(clip ? "clip" : "clamp", W, H, o[2], 1);
            }

    for (int am = 0; am < 2; ++am)
        for (int fl = 0; fl < 2; ++fl) {
            svo_reproject(W, H, f.z, f.nx, f.ny, f.nz, NULL, f.mvx, f.mvy,
                          f.pz, f.pnx, f.pny, f.pnz, NULL, f.hr, f.hg, f.hb,
                          f.hm1, f.hm2, f.hn, 0.05, 0.9, 0, o[8], o[9], o[10],
                          o[11], o[12], on, ov);
            canary(n, o[0], o[1], o[2]);
            canary(n, o[3], o[4], NULL);
            svo_blend(n, f.cr, f.cg, f.cb, f.z, o[8], o[9], o[10], o[11],
                      o[12], on, ov, 0.2, 0.2, am ? f.amap : NULL, 32,
                      fl ? HALF_OUT : 0, o[0], o[1], o[2], o[3], o[4], on2);
            ++g_cases;
            check_written("blend", W, H, o[0], 1);
            check_written("blend m2", W, H, o[4], 1);
            check_iwritten("blend n", W, H, on2, 0, 32);
        }

    for (int flags = 0; flags < 16; ++flags)
        for (int of = 0; of < 2; ++of) {
            canary(n, o[0], o[1], o[2]);
            canary(n, o[3], o[4], NULL);
            int rc = svo_temporal(
                W, H, f.cr, f.cg, f.cb, f.z, f.nx, f.ny, f.nz, f.id, f.mvx,
                f.mvy, f.pz, f.pnx, f.pny, f.pnz, f.pid, f.hr, f.hg, f.hb,
                f.hm1, f.hm2, f.hn, 0.2, 0.2, 1.0, 0.05, 0.9, 1.0, 32, flags,
                of ? HALF_OUT : 0, (flags & 1) ? f.amap : NULL, o[0], o[1],
                o[2], o[3], o[4], on);
            ++g_cases;
            if (rc != 0) {
                fprintf(stderr, "FAIL temporal rc %d\n", rc);
                g_fail = 1;
            }
            check_written("temporal", W, H, o[0], 1);
            check_iwritten("temporal n", W, H, on, 0, 32);
        }

    /* temporal results feed the variance and the a-trous levels */
    double *m1 = o[3], *m2 = o[4];
    double *var = plane(n);
    for (int radius = 0; radius <= 3; ++radius)
        for (int mh = 1; mh <= 4; mh += 3) {
            canary(n, var, NULL, NULL);
            svo_variance(W, H, m1, m2, on, f.z, f.dzdx, f.dzdy, f.nx, f.ny,
                         f.nz, 1.0, 128.0, 1e-2, mh, radius, var);
            ++g_cases;
            check_written("variance", W, H, var, 1);
        }

    static const int steps[] = {1, 2, 4, 8, 16, 32, 64};
    double *sh[3] = {plane(n), plane(n), plane(n)};
    for (size_t si = 0; si < sizeof steps / sizeof steps[0]; ++si)
        for (int flags = 0; flags < 8; ++flags)
            for (int k = 0; k < 2; ++k) {
                int step = steps[si];
                const double *kap = k ? f.kappa : NULL;
                double *vo = (flags & 1) ? NULL : o[5];
                canary(n, o[6], o[7], o[8]);
                canary(n, vo, NULL, NULL);
                svo_atrous(W, H, o[0], o[1], o[2], var, f.z, f.dzdx, f.dzdy,
                           f.nx, f.ny, f.nz, kap, step, 1.0, 128.0, 4.0, 1e-2,
                           1e-10, 1.0, flags, o[6], o[7], o[8], vo);
                ++g_cases;
                check_written("atrous", W, H, o[6], 1);
                check_written("atrous b", W, H, o[8], 1);
                if (vo)
                    check_written("atrous var", W, H, vo, 1);
                canary(n, o[6], o[7], o[8]);
                canary(n, sh[0], sh[1], sh[2]);
                canary(n, vo, NULL, NULL);
                svo_atrous_sep(W, H, o[0], o[1], o[2], var, f.z, f.dzdx,
                               f.dzdy, f.nx, f.ny, f.nz, kap, step, 1.0, 128.0,
                               4.0, 1e-2, 1e-10, 1.0, flags, sh[0], sh[1],
                               sh[2], o[6], o[7], o[8], vo);
                ++g_cases;
                check_written("atrous_sep h", W, H, sh[0], 1);
                check_written("atrous_sep", W, H, o[7], 1);
                if (vo)
                    check_written("atrous_sep var", W, H, vo, 1);
            }

    for (int i = 0; i < 3; ++i)
        free(sh[i]);
    free(var);
    for (int i = 0; i < 13; ++i)
        free(o[i]);
    free(on);
    free(ov);
    free(on2);
    frame_free(&f);
}

int main(void)
{
    static const int sizes[][2] = {{1, 1}, {1, 9}, {9, 1}, {2, 2}, {5, 3},
                                   {3, 5}, {33, 17}, {70, 2}, {2, 70}};
    if (svo_version() <= 0) {
        fprintf(stderr, "FAIL version\n");
        return 1;
    }
    case_half();
    for (int threads = 1; threads <= 3; threads += 2) {
        svo_set_threads(threads);
        for (size_t i = 0; i < sizeof sizes / sizeof sizes[0]; ++i)
            for (int hostile = 0; hostile < 2; ++hostile)
                case_frame(sizes[i][0], sizes[i][1], hostile);
    }
    if (svo_threads() < 1) {
        fprintf(stderr, "FAIL threads\n");
        return 1;
    }
    if (g_fail)
        return 1;
    printf("selftest ok %ld\n", g_cases);
    return 0;
}
