/*
 * ebof_oracle.c -- plain CPU oracle of the event-based optical-flow hot path
 * of arXiv 2112.10591 (Brebion, Moreau, Davoine).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the GPU library.  Written for obviousness, not speed: every function
 * follows the definition or the algorithm of the passage it cites, in double
 * precision, single-threaded.
 *
 * Build: cc -O2 -ffp-contract=off -std=c99 -fPIC -shared ebof_oracle.c -lm
 * (no FMA contraction, so every product and sum is rounded as written).
 */
#include "ebof_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Section III-A, accumulation: an edge image is a binary matrix telling    */
/* whether a pixel produced at least one event during the window; polarity */
/* plays no part.  Window reading: half-open [t0, t0 + dt).                 */
/* ------------------------------------------------------------------------ */
int64_t oref_edge_image(int32_t W, int32_t H, const uint16_t *x,
                        const uint16_t *y, const int64_t *t, int64_t n,
                        int64_t t0, int64_t dt, uint8_t *E)
{
    int64_t binned = 0;
    memset(E, 0, (size_t)W * (size_t)H);
    for (int64_t i = 0; i < n; i++) {
        if (t[i] < t0 || t[i] >= t0 + dt)
            continue;
        if ((int32_t)x[i] >= W || (int32_t)y[i] >= H)
            continue;
        E[(size_t)y[i] * (size_t)W + x[i]] = 1;
        binned++;
    }
    return n - binned;
}

/* 1 when (x, y) lies inside the image and is an edge pixel; pixels outside
 * the image count as non-edges. */
static int edge_at(const uint8_t *E, int32_t W, int32_t H, int32_t x,
                   int32_t y)
{
    if (x < 0 || y < 0 || x >= W || y >= H)
        return 0;
    return E[(size_t)y * (size_t)W + x] != 0;
}

static int four_neighbours(const uint8_t *E, int32_t W, int32_t H, int32_t x,
                           int32_t y)
{
    return edge_at(E, W, H, x - 1, y) + edge_at(E, W, H, x + 1, y) +
           edge_at(E, W, H, x, y - 1) + edge_at(E, W, H, x, y + 1);
}

/* Algorithm 1: E_d starts as a copy of E; every edge pixel of E whose count
 * of edge 4-neighbours (counted in E, never in E_d) is below N_d is removed. */
void oref_denoise(int32_t W, int32_t H, const uint8_t *E, int32_t n_d,
                  uint8_t *Ed)
{
    memcpy(Ed, E, (size_t)W * (size_t)H);
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            if (!edge_at(E, W, H, x, y))
                continue;
            if (four_neighbours(E, W, H, x, y) < n_d)
                Ed[(size_t)y * W + x] = 0;
        }
}

/* Algorithm 2: E_df starts as a copy of E_d; every non-edge pixel of E_d
 * whose count of edge 4-neighbours (counted in E_d) is at least N_f becomes
 * an edge. */
void oref_fill(int32_t W, int32_t H, const uint8_t *Ed, int32_t n_f,
               uint8_t *Edf)
{
    memcpy(Edf, Ed, (size_t)W * (size_t)H);
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            if (edge_at(Ed, W, H, x, y))
                continue;
            if (four_neighbours(Ed, W, H, x, y) >= n_f)
                Edf[(size_t)y * W + x] = 1;
        }
}

/* ------------------------------------------------------------------------ */
/* Section III-C: d_Euc is the Euclidean distance to the closest edge pixel. */
/* The oracle keeps its square, an integer.                                 */
/* ------------------------------------------------------------------------ */
int32_t oref_edt_brute_at(int32_t W, int32_t H, const uint8_t *E, int32_t px,
                          int32_t py)
{
    int64_t best = INT32_MAX;
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            if (!E[(size_t)y * W + x])
                continue;
            int64_t dx = x - px, dy = y - py;
            int64_t d = dx * dx + dy * dy;
            if (d < best)
                best = d;
        }
    return (int32_t)best;
}

void oref_edt_brute(int32_t W, int32_t H, const uint8_t *E, int32_t *D2)
{
    /* list the edge pixels once, then take the minimum for every pixel */
    int64_t ne = 0;
    for (int64_t i = 0; i < (int64_t)W * H; i++)
        ne += E[i] != 0;
    int32_t *ex = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne + 1));
    int32_t *ey = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne + 1));
    int64_t k = 0;
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++)
            if (E[(size_t)y * W + x]) {
                ex[k] = x;
                ey[k] = y;
                k++;
            }
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            int64_t best = INT32_MAX;
            for (int64_t i = 0; i < ne; i++) {
                int64_t dx = ex[i] - x, dy = ey[i] - y;
                int64_t d = dx * dx + dy * dy;
                if (d < best)
                    best = d;
            }
            D2[(size_t)y * W + x] = (int32_t)best;
        }
    free(ex);
    free(ey);
}

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0))
        q -= 1;
    return q;
}

/* Exact separable squared distance transform (the separable scheme of the
 * distance-transform literature that Section III-C builds on):
 *   phase 1, per column x: g(x, y) = min |y - y'| over edge pixels (x, y');
 *   phase 2, per row y:    D2(x, y) = min_x' (x - x')^2 + g(x', y)^2,
 * the second phase as the lower envelope of the parabolas
 * F_x'(x) = (x - x')^2 + g(x', y)^2 over the columns x' that hold an edge.
 * All integer arithmetic, so the result is exact. */
void oref_edt_separable(int32_t W, int32_t H, const uint8_t *E, int32_t *D2)
{
    const int64_t INF = -1; /* marks "no edge in this column" */
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)W * (size_t)H);
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * (size_t)W);
    int64_t *site = (int64_t *)malloc(sizeof(int64_t) * (size_t)W);
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)W);

    /* phase 1: two sweeps per column */
    for (int32_t x = 0; x < W; x++) {
        int64_t last = INF;
        for (int32_t y = 0; y < H; y++) {
            if (E[(size_t)y * W + x])
                last = y;
            g[(size_t)y * W + x] = (last == INF) ? INF : (y - last);
        }
        last = INF;
        for (int32_t y = H - 1; y >= 0; y--) {
            if (E[(size_t)y * W + x])
                last = y;
            if (last != INF) {
                int64_t d = last - y;
                int64_t *gp = &g[(size_t)y * W + x];
                if (*gp == INF || d < *gp)
                    *gp = d;
            }
        }
    }

    /* phase 2: lower envelope per row */
    for (int32_t y = 0; y < H; y++) {
        int64_t q = -1; /* index of the last parabola in the envelope */
        for (int32_t x = 0; x < W; x++) {
            int64_t gv = g[(size_t)y * W + x];
            f[x] = (gv == INF) ? INF : gv * gv;
        }
        for (int64_t u = 0; u < W; u++) {
            if (f[u] == INF)
                continue;
            /* drop parabolas that u beats at the start of their segment */
            while (q >= 0) {
                int64_t s = site[q], at = start[q];
                int64_t fs = (at - s) * (at - s) + f[s];
                int64_t fu = (at - u) * (at - u) + f[u];
                if (fs > fu)
                    q--;
                else
                    break;
            }
            if (q < 0) {
                q = 0;
                site[0] = u;
                start[0] = 0;
            } else {
                /* first integer x where parabola u is strictly below site[q]:
                 * (x-u)^2+f(u) < (x-s)^2+f(s)  <=>  x > sep */
                int64_t s = site[q];
                int64_t sep = floor_div(u * u - s * s + f[u] - f[s], 2 * (u - s));
                int64_t w = sep + 1;
                if (w < W) {
                    q++;
                    site[q] = u;
                    start[q] = w;
                }
            }
        }
        if (q < 0) { /* no edge pixel anywhere in the image */
            for (int32_t x = 0; x < W; x++)
                D2[(size_t)y * W + x] = INT32_MAX;
            continue;
        }
        for (int64_t x = W - 1; x >= 0; x--) {
            int64_t s = site[q];
            int64_t d = (x - s) * (x - s) + f[s];
            D2[(size_t)y * W + x] = (int32_t)d;
            if (x == start[q])
                q--;
        }
    }
    free(g);
    free(f);
    free(site);
    free(start);
}

/* Equation (1): d_exp = 1 - exp(-d_Euc / alpha). */
void oref_surface(int64_t n, const int32_t *D2, double alpha, float *S)
{
    for (int64_t i = 0; i < n; i++) {
        double d = sqrt((double)D2[i]);
        S[i] = (float)(1.0 - exp(-d / alpha));
    }
}

/* Ablation surfaces (Sec. IV-B): the proposed inverse exponential, the plain
 * distance, the distance bounded at d_sat (6 px in the paper, which equals
 * alpha ln 255 by eq. 3) and its logarithm. */
void oref_surface_kind(int64_t n, const int32_t *D2, double alpha, int32_t kind,
                       float *S)
{
    double d_sat = alpha * log(255.0);
    for (int64_t i = 0; i < n; i++) {
        double d = sqrt((double)D2[i]);
        double v;
        if (kind == 1)
            v = d;
        else if (kind == 2)
            v = d < d_sat ? d : d_sat;
        else if (kind == 3)
            v = log(d + 1.0);
        else
            v = 1.0 - exp(-d / alpha);
        S[i] = (float)v;
    }
}

/* ------------------------------------------------------------------------ */
/* Evaluation metrics (Sec. IV): average endpoint error, outliers, and the   */
/* flow warp loss.                                                           */
/* ------------------------------------------------------------------------ */
int64_t oref_flow_errors(int64_t n, const double *u, const double *v,
                         const uint8_t *mask, double *aee, double *outliers)
{
    int64_t cnt = 0, out = 0;
    double sum = 0.0;
    for (int64_t i = 0; i < n; i++) {
        if (mask && !mask[i])
            continue;
        double ex = v[i] - u[i], ey = v[n + i] - u[n + i];
        double e = sqrt(ex * ex + ey * ey);
        double m = sqrt(v[i] * v[i] + v[n + i] * v[n + i]);
        sum += e;
        if (e > 3.0 && e > 0.05 * m)
            out++;
        cnt++;
    }
    *aee = cnt ? sum / (double)cnt : 0.0;
    *outliers = cnt ? (double)out / (double)cnt : 0.0;
    return cnt;
}

static double image_variance(const double *I, int64_t N)
{
    double s = 0.0;
    for (int64_t i = 0; i < N; i++)
        s += I[i];
    double m = s / (double)N, q = 0.0;
    for (int64_t i = 0; i < N; i++)
        q += (I[i] - m) * (I[i] - m);
    return q / (double)N;
}

double oref_fwl(int32_t W, int32_t H, const uint16_t *x, const uint16_t *y,
                const int64_t *t, const int8_t *pol, int64_t n, int64_t t0,
                int64_t dt, const double *flow, double *var_comp,
                double *var_uncomp)
{
    size_t N = (size_t)W * H;
    double *Ic = (double *)calloc(N, sizeof(double));
    double *Iu = (double *)calloc(N, sizeof(double));
    for (int64_t e = 0; e < n; e++) {
        if (t[e] < t0 || t[e] >= t0 + dt || x[e] >= W || y[e] >= H)
            continue;
        double w = pol ? (pol[e] < 0 ? -1.0 : 1.0) : 1.0;
        size_t p = (size_t)y[e] * W + x[e];
        Iu[p] += w;
        double tau = (double)(t[e] - t0) / (double)dt;
        double sx = x[e] - flow[p] * tau, sy = y[e] - flow[N + p] * tau;
        double fx = floor(sx), fy = floor(sy);
        double ax = sx - fx, ay = sy - fy;
        for (int32_t j = 0; j < 2; j++)
            for (int32_t i = 0; i < 2; i++) {
                double X = fx + i, Y = fy + j;
                if (X < 0 || X >= W || Y < 0 || Y >= H)
                    continue;
                double b = (i ? ax : 1.0 - ax) * (j ? ay : 1.0 - ay);
                Ic[(size_t)Y * W + (size_t)X] += w * b;
            }
    }
    double vc = image_variance(Ic, (int64_t)N), vu = image_variance(Iu, (int64_t)N);
    free(Ic);
    free(Iu);
    *var_comp = vc;
    *var_uncomp = vu;
    return vu > 0.0 ? vc / vu : 0.0;
}

/* Adaptive windows (the Conclusion's adaptive accumulation time, with the
 * area event count as the rule): the sensor is tiled by squares of side
 * `area` pixels from (0, 0); scanning a time-ordered stream from event i0,
 * each on-sensor event counts for its square, and the window ends right after
 * the event that brings some square to k_events.  Returns that end (one past
 * the event), or n when no square reaches k_events.  Events off the sensor
 * are skipped (they count for no square). */
int64_t oref_window_end_area(int32_t W, int32_t H, const uint16_t *x,
                             const uint16_t *y, int64_t n, int64_t i0,
                             int32_t area, int32_t k_events)
{
    int32_t ax = (W + area - 1) / area, ay = (H + area - 1) / area;
    int32_t *cnt = (int32_t *)calloc((size_t)ax * ay, sizeof(int32_t));
    int64_t end = n;
    for (int64_t e = i0; e < n; e++) {
        if (x[e] >= W || y[e] >= H)
            continue;
        int32_t m = (y[e] / area) * ax + x[e] / area;
        if (++cnt[m] >= k_events) {
            end = e + 1;
            break;
        }
    }
    free(cnt);
    return end;
}

/* ------------------------------------------------------------------------ */
/* Gaussian pyramid of a surface: binomial 5-tap blur then keep every second */
/* pixel, reflect-101 border.                                               */
/* ------------------------------------------------------------------------ */
static int32_t reflect101(int32_t i, int32_t n)
{
    if (i < 0)
        return -i;
    if (i >= n)
        return 2 * n - 2 - i;
    return i;
}

void oref_pyr_down(int32_t W, int32_t H, const float *in, float *out)
{
    static const double k[5] = {1.0, 4.0, 6.0, 4.0, 1.0};
    int32_t Wo = (W + 1) / 2, Ho = (H + 1) / 2;
    for (int32_t Y = 0; Y < Ho; Y++)
        for (int32_t X = 0; X < Wo; X++) {
            double acc = 0.0;
            for (int32_t j = -2; j <= 2; j++)
                for (int32_t i = -2; i <= 2; i++) {
                    int32_t xx = reflect101(2 * X + i, W);
                    int32_t yy = reflect101(2 * Y + j, H);
                    acc += k[i + 2] * k[j + 2] * (double)in[(size_t)yy * W + xx];
                }
            out[(size_t)Y * Wo + X] = (float)(acc / 256.0);
        }
}

/* ------------------------------------------------------------------------ */
/* Frame-based flow between consecutive surfaces (Section III-D allows any   */
/* frame-based method): dense inverse search.  Per level, coarse to fine:    */
/* a regular grid of ps x ps patches at the given stride, each refined by    */
/* inverse-compositional Lucas-Kanade (translation only), reset to its       */
/* initial value when it moved more than ps, then densified into a per-pixel */
/* flow by a weighted mean of the patches covering each pixel.              */
/* ------------------------------------------------------------------------ */
static double at_clamped(const float *I, int32_t W, int32_t H, int64_t x,
                         int64_t y)
{
    if (x < 0)
        x = 0;
    if (x > W - 1)
        x = W - 1;
    if (y < 0)
        y = 0;
    if (y > H - 1)
        y = H - 1;
    return (double)I[(size_t)y * W + x];
}

/* bilinear interpolation at (sx, sy) with replicated borders: the four
 * neighbouring sample indices are clamped into the image */
static double bilinear(const float *I, int32_t W, int32_t H, double sx,
                       double sy)
{
    double fx = floor(sx), fy = floor(sy);
    double ax = sx - fx, ay = sy - fy;
    /* indices beyond the border all clamp to the border, so the integer part
     * can be limited before conversion without changing the result */
    if (fx < -2.0)
        fx = -2.0;
    if (fx > W + 2.0)
        fx = W + 2.0;
    if (fy < -2.0)
        fy = -2.0;
    if (fy > H + 2.0)
        fy = H + 2.0;
    int64_t x0 = (int64_t)fx, y0 = (int64_t)fy;
    double i00 = at_clamped(I, W, H, x0, y0);
    double i10 = at_clamped(I, W, H, x0 + 1, y0);
    double i01 = at_clamped(I, W, H, x0, y0 + 1);
    double i11 = at_clamped(I, W, H, x0 + 1, y0 + 1);
    return (1.0 - ay) * ((1.0 - ax) * i00 + ax * i10) +
           ay * ((1.0 - ax) * i01 + ax * i11);
}

int64_t oref_patch_count(int32_t W, int32_t H, int32_t ps, int32_t stride)
{
    if (W < ps || H < ps || ps < 1 || stride < 1)
        return 0;
    int64_t nx = (W - ps + stride - 1) / stride + 1;
    int64_t ny = (H - ps + stride - 1) / stride + 1;
    return nx * ny;
}

/* origin of patch k along an axis of n pixels: k*stride, the last one
 * clamped so that it ends on the border */
static int32_t patch_origin(int32_t k, int32_t stride, int32_t n, int32_t ps)
{
    int32_t o = k * stride;
    if (o > n - ps)
        o = n - ps;
    return o;
}

/* Densification: U(x) = sum_i w_i u_i / sum_i w_i over the patches i that
 * contain x, w_i = 1 / max(1, 255 |I1(x + u_i) - I0(x)|).  The 255 puts the
 * [0,1] surface on the 8-bit scale that the weight's unit threshold assumes
 * (the same 8-bit coding eq. (3) takes for its saturation gap).  Every pixel
 * lies in at least one patch (the last origin of each axis is clamped to the
 * border), so the denominator is positive. */
void oref_densify(int32_t W, int32_t H, const float *I0, const float *I1,
                  int32_t ps, int32_t stride, const double *pu,
                  double *U /* 2*W*H */)
{
    int32_t nx = (W - ps + stride - 1) / stride + 1;
    int32_t ny = (H - ps + stride - 1) / stride + 1;
    size_t N = (size_t)W * H;
    double *acc_w = (double *)calloc(N, sizeof(double));
    double *acc_u = (double *)calloc(N, sizeof(double));
    double *acc_v = (double *)calloc(N, sizeof(double));
    for (int32_t ky = 0; ky < ny; ky++)
        for (int32_t kx = 0; kx < nx; kx++) {
            int32_t ox = patch_origin(kx, stride, W, ps);
            int32_t oy = patch_origin(ky, stride, H, ps);
            double u = pu[2 * ((size_t)ky * nx + kx)];
            double v = pu[2 * ((size_t)ky * nx + kx) + 1];
            for (int32_t j = 0; j < ps; j++)
                for (int32_t i = 0; i < ps; i++) {
                    int32_t x = ox + i, y = oy + j;
                    double d = bilinear(I1, W, H, x + u, y + v) -
                               (double)I0[(size_t)y * W + x];
                    double s = 255.0 * fabs(d);
                    double w = 1.0 / (s > 1.0 ? s : 1.0);
                    size_t p = (size_t)y * W + x;
                    acc_w[p] += w;
                    acc_u[p] += w * u;
                    acc_v[p] += w * v;
                }
        }
    for (size_t p = 0; p < N; p++) {
        U[p] = acc_u[p] / acc_w[p];
        U[N + p] = acc_v[p] / acc_w[p];
    }
    free(acc_w);
    free(acc_u);
    free(acc_v);
}

/* Coarse-to-fine start of a level: a patch starts from twice the coarser
 * level's dense flow Uc (Wc x Hc, two planes) at the coarser pixel nearest
 * to the patch centre, i.e. at (floor((o_x + ps/2) / 2), floor((o_y + ps/2)
 * / 2)), clamped into the coarser image. */
void oref_patch_init_coarser(int32_t W, int32_t H, int32_t ps, int32_t stride,
                             const double *Uc, int32_t Wc, int32_t Hc,
                             double *u0)
{
    int32_t nx = (W - ps + stride - 1) / stride + 1;
    int32_t ny = (H - ps + stride - 1) / stride + 1;
    for (int32_t ky = 0; ky < ny; ky++)
        for (int32_t kx = 0; kx < nx; kx++) {
            int32_t cx = (patch_origin(kx, stride, W, ps) + ps / 2) / 2;
            int32_t cy = (patch_origin(ky, stride, H, ps) + ps / 2) / 2;
            if (cx > Wc - 1)
                cx = Wc - 1;
            if (cy > Hc - 1)
                cy = Hc - 1;
            size_t k = (size_t)ky * nx + kx;
            u0[2 * k] = 2.0 * Uc[(size_t)cy * Wc + cx];
            u0[2 * k + 1] = 2.0 * Uc[(size_t)Wc * Hc + (size_t)cy * Wc + cx];
        }
}

/* Warm start of the coarsest level (level `level` of a W0 x H0 sensor) from
 * the previous window pair's dense level-0 flow Up (the temporal
 * propagation Sec. III-D values in its flow method, reduced to a prediction
 * of constant motion): a patch starts from Up at the level-0 pixel under
 * its centre, (o + ps/2) * 2^level clamped into the sensor, divided by
 * 2^level (a displacement of level 0 spans 2^level times fewer pixels
 * there). */
void oref_patch_init_previous(int32_t W, int32_t H, int32_t level, int32_t ps,
                              int32_t stride, const double *Up, int32_t W0,
                              int32_t H0, double *u0)
{
    int32_t nx = (W - ps + stride - 1) / stride + 1;
    int32_t ny = (H - ps + stride - 1) / stride + 1;
    double scale = 1.0;
    for (int32_t l = 0; l < level; l++)
        scale *= 2.0;
    for (int32_t ky = 0; ky < ny; ky++)
        for (int32_t kx = 0; kx < nx; kx++) {
            int64_t px = (int64_t)(patch_origin(kx, stride, W, ps) + ps / 2) << level;
            int64_t py = (int64_t)(patch_origin(ky, stride, H, ps) + ps / 2) << level;
            if (px > W0 - 1)
                px = W0 - 1;
            if (py > H0 - 1)
                py = H0 - 1;
            size_t k = (size_t)ky * nx + kx;
            u0[2 * k] = Up[(size_t)py * W0 + px] / scale;
            u0[2 * k + 1] = Up[(size_t)W0 * H0 + (size_t)py * W0 + px] / scale;
        }
}

/* Patch inverse search on one level: every patch starts from its u0,
 * takes `iters` inverse-compositional Lucas-Kanade steps (translation only)
 * with the Hessian regularised by lambda I, and returns to u0 when it moved
 * more than ps (Euclidean) from it. */
void oref_dis_level(int32_t W, int32_t H, const float *I0, const float *I1,
                    int32_t ps, int32_t stride, int32_t iters, double lambda,
                    const double *u0, double *pu)
{
    int32_t nx = (W - ps + stride - 1) / stride + 1;
    int32_t ny = (H - ps + stride - 1) / stride + 1;
    double *gx = (double *)malloc(sizeof(double) * (size_t)ps * ps);
    double *gy = (double *)malloc(sizeof(double) * (size_t)ps * ps);
    double *T = (double *)malloc(sizeof(double) * (size_t)ps * ps);
    for (int32_t ky = 0; ky < ny; ky++)
        for (int32_t kx = 0; kx < nx; kx++) {
            int32_t ox = patch_origin(kx, stride, W, ps);
            int32_t oy = patch_origin(ky, stride, H, ps);
            size_t k = (size_t)ky * nx + kx;
            double su = u0 ? u0[2 * k] : 0.0, sv = u0 ? u0[2 * k + 1] : 0.0;

            /* template, its gradient (central differences, replicated
             * border) and the Gauss-Newton Hessian H = sum g g^T */
            double hxx = 0.0, hxy = 0.0, hyy = 0.0;
            for (int32_t j = 0; j < ps; j++)
                for (int32_t i = 0; i < ps; i++) {
                    int32_t x = ox + i, y = oy + j;
                    int32_t q = j * ps + i;
                    T[q] = (double)I0[(size_t)y * W + x];
                    gx[q] = 0.5 * (at_clamped(I0, W, H, x + 1, y) -
                                   at_clamped(I0, W, H, x - 1, y));
                    gy[q] = 0.5 * (at_clamped(I0, W, H, x, y + 1) -
                                   at_clamped(I0, W, H, x, y - 1));
                    hxx += gx[q] * gx[q];
                    hxy += gx[q] * gy[q];
                    hyy += gy[q] * gy[q];
                }
            double a = hxx + lambda, c = hyy + lambda, bb = hxy;
            double det = a * c - bb * bb;

            /* inverse-compositional iterations, a fixed number of them */
            double u = su, v = sv;
            for (int32_t it = 0; it < iters; it++) {
                double bx = 0.0, by = 0.0;
                for (int32_t j = 0; j < ps; j++)
                    for (int32_t i = 0; i < ps; i++) {
                        int32_t q = j * ps + i;
                        double r = bilinear(I1, W, H, ox + i + u, oy + j + v) - T[q];
                        bx += gx[q] * r;
                        by += gy[q] * r;
                    }
                /* (H + lambda I) d = b, solved by the 2x2 inverse */
                double dx = (c * bx - bb * by) / det;
                double dy = (a * by - bb * bx) / det;
                u -= dx;
                v -= dy;
            }
            /* outlier reset: a patch that moved more than its size
             * returns to its initial displacement */
            double mu = u - su, mv = v - sv;
            if (sqrt(mu * mu + mv * mv) > (double)ps) {
                u = su;
                v = sv;
            }
            pu[2 * k] = u;
            pu[2 * k + 1] = v;
        }
    free(gx);
    free(gy);
    free(T);
}

/* ------------------------------------------------------------------------ */
/* Variational refinement of a dense flow (the third stage of dense inverse  */
/* search): a few fixed-point iterations of the linearised robust energy     */
/*   sum_x delta Psi(E_c) + gamma Psi(E_g) + alpha Psi(|grad(u)|^2 +          */
/*         |grad(v)|^2),  Psi(s^2) = sqrt(s^2 + eps^2),                       */
/* E_c the brightness-constancy and E_g the gradient-constancy residual of   */
/* the flow increment, each solved by red-black block SOR.                   */
/* ------------------------------------------------------------------------ */
static double px_clamped(const double *f, int32_t W, int32_t H, int64_t x,
                         int64_t y)
{
    if (x < 0)
        x = 0;
    if (x >= W)
        x = W - 1;
    if (y < 0)
        y = 0;
    if (y >= H)
        y = H - 1;
    return f[(size_t)y * W + x];
}

/* central differences along x and y, replicated border */
static void grad(const double *f, int32_t W, int32_t H, double *fx, double *fy)
{
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            size_t p = (size_t)y * W + x;
            fx[p] = 0.5 * (px_clamped(f, W, H, x + 1, y) - px_clamped(f, W, H, x - 1, y));
            fy[p] = 0.5 * (px_clamped(f, W, H, x, y + 1) - px_clamped(f, W, H, x, y - 1));
        }
}

static double robust_weight(double s2)
{
    const double eps = 1e-3;
    return 1.0 / sqrt(s2 + eps * eps);
}

void oref_var_refine(int32_t W, int32_t H, const float *I0f, const float *I1f,
                     double *U, int32_t outer, int32_t inner, double alpha,
                     double gamma, double delta, double omega)
{
    size_t N = (size_t)W * H;
    /* images on the 8-bit scale the weights assume */
    double *I0 = (double *)malloc(sizeof(double) * N);
    double *I1w = (double *)malloc(sizeof(double) * N);
    double *A = (double *)malloc(sizeof(double) * N);
    double *d[14];
    for (int i = 0; i < 14; i++)
        d[i] = (double *)malloc(sizeof(double) * N);
    double *gx0 = d[0], *gy0 = d[1], *gx1 = d[2], *gy1 = d[3];
    double *Ix = d[4], *Iy = d[5], *Ixx = d[6], *Ixy = d[7], *Iyx = d[8], *Iyy = d[9];
    double *du = d[10], *dv = d[11], *s = d[12], *tmp = d[13];
    double *It = (double *)malloc(sizeof(double) * N);
    double *Ixt = (double *)malloc(sizeof(double) * N);
    double *Iyt = (double *)malloc(sizeof(double) * N);
    double *a11 = (double *)malloc(sizeof(double) * N);
    double *a12 = (double *)malloc(sizeof(double) * N);
    double *a22 = (double *)malloc(sizeof(double) * N);
    double *b1 = (double *)malloc(sizeof(double) * N);
    double *b2 = (double *)malloc(sizeof(double) * N);
    (void)tmp;
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            size_t p = (size_t)y * W + x;
            I0[p] = 255.0 * (double)I0f[p];
            I1w[p] = 255.0 * bilinear(I1f, W, H, x + U[p], y + U[N + p]);
            A[p] = 0.5 * (I0[p] + I1w[p]);
            It[p] = I1w[p] - I0[p];
        }
    /* first derivatives of both images and of their average, then the
     * second derivatives of the average; the temporal change of the
     * gradient is the warped image's gradient minus the reference's */
    grad(I0, W, H, gx0, gy0);
    grad(I1w, W, H, gx1, gy1);
    grad(A, W, H, Ix, Iy);
    grad(Ix, W, H, Ixx, Ixy);
    grad(Iy, W, H, Iyx, Iyy);
    for (size_t p = 0; p < N; p++) {
        Ixt[p] = gx1[p] - gx0[p];
        Iyt[p] = gy1[p] - gy0[p];
        Ixy[p] = 0.5 * (Ixy[p] + Iyx[p]); /* the mixed derivative, symmetrised */
        du[p] = 0.0;
        dv[p] = 0.0;
    }
    for (int32_t o = 0; o < outer; o++) {
        /* weights at the current increment (lagged) */
        for (int32_t y = 0; y < H; y++)
            for (int32_t x = 0; x < W; x++) {
                size_t p = (size_t)y * W + x;
                double c = It[p] + (Ix[p] * du[p] + Iy[p] * dv[p]);
                double g1 = Ixt[p] + (Ixx[p] * du[p] + Ixy[p] * dv[p]);
                double g2 = Iyt[p] + (Ixy[p] * du[p] + Iyy[p] * dv[p]);
                double wc = delta * robust_weight(c * c);
                double wg = gamma * robust_weight(g1 * g1 + g2 * g2);
                a11[p] = wc * Ix[p] * Ix[p] + wg * (Ixx[p] * Ixx[p] + Ixy[p] * Ixy[p]);
                a12[p] = wc * (Ix[p] * Iy[p]) + wg * (Ixx[p] * Ixy[p] + Ixy[p] * Iyy[p]);
                a22[p] = wc * Iy[p] * Iy[p] + wg * (Ixy[p] * Ixy[p] + Iyy[p] * Iyy[p]);
                b1[p] = wc * Ix[p] * It[p] + wg * (Ixx[p] * Ixt[p] + Ixy[p] * Iyt[p]);
                b2[p] = wc * Iy[p] * It[p] + wg * (Ixy[p] * Ixt[p] + Iyy[p] * Iyt[p]);
                /* smoothness weight of the total flow u + du, v + dv */
                double ux = 0.5 * ((px_clamped(U, W, H, x + 1, y) + px_clamped(du, W, H, x + 1, y)) -
                                   (px_clamped(U, W, H, x - 1, y) + px_clamped(du, W, H, x - 1, y)));
                double uy = 0.5 * ((px_clamped(U, W, H, x, y + 1) + px_clamped(du, W, H, x, y + 1)) -
                                   (px_clamped(U, W, H, x, y - 1) + px_clamped(du, W, H, x, y - 1)));
                double vx = 0.5 * ((px_clamped(U + N, W, H, x + 1, y) + px_clamped(dv, W, H, x + 1, y)) -
                                   (px_clamped(U + N, W, H, x - 1, y) + px_clamped(dv, W, H, x - 1, y)));
                double vy = 0.5 * ((px_clamped(U + N, W, H, x, y + 1) + px_clamped(dv, W, H, x, y + 1)) -
                                   (px_clamped(U + N, W, H, x, y - 1) + px_clamped(dv, W, H, x, y - 1)));
                /* (summed so that swapping the axes, u and v, swaps nothing) */
                s[p] = alpha * robust_weight((ux * ux + vy * vy) + (uy * uy + vx * vx));
            }
        /* red-black block SOR: pixels with x + y even, then odd; each solves
         * its 2x2 system with the neighbours' current increments and relaxes
         * towards the solution */
        for (int32_t it = 0; it < inner; it++)
            for (int32_t colour = 0; colour < 2; colour++)
                for (int32_t y = 0; y < H; y++)
                    for (int32_t x = 0; x < W; x++) {
                        if (((x + y) & 1) != colour)
                            continue;
                        size_t p = (size_t)y * W + x;
                        /* the four neighbours (absent ones weigh 0), added
                         * as (left + right) + (up + down) */
                        double w[4] = {0.0, 0.0, 0.0, 0.0}, tu[4] = {0.0, 0.0, 0.0, 0.0},
                               tv[4] = {0.0, 0.0, 0.0, 0.0};
                        const int32_t nx[4] = {x - 1, x + 1, x, x};
                        const int32_t ny[4] = {y, y, y - 1, y + 1};
                        for (int k = 0; k < 4; k++) {
                            if (nx[k] < 0 || nx[k] >= W || ny[k] < 0 || ny[k] >= H)
                                continue;
                            size_t q = (size_t)ny[k] * W + nx[k];
                            w[k] = 0.5 * (s[p] + s[q]);
                            tu[k] = w[k] * ((U[q] - U[p]) + du[q]);
                            tv[k] = w[k] * ((U[N + q] - U[N + p]) + dv[q]);
                        }
                        double sw = (w[0] + w[1]) + (w[2] + w[3]);
                        double ru = (tu[0] + tu[1]) + (tu[2] + tu[3]);
                        double rv = (tv[0] + tv[1]) + (tv[2] + tv[3]);
                        double m11 = a11[p] + sw, m22 = a22[p] + sw, m12 = a12[p];
                        double r1 = ru - b1[p], r2 = rv - b2[p];
                        double det = m11 * m22 - m12 * m12;
                        double su = (m22 * r1 - m12 * r2) / det;
                        double sv = (m11 * r2 - m12 * r1) / det;
                        du[p] = (1.0 - omega) * du[p] + omega * su;
                        dv[p] = (1.0 - omega) * dv[p] + omega * sv;
                    }
    }
    for (size_t p = 0; p < N; p++) {
        U[p] += du[p];
        U[N + p] += dv[p];
    }
    free(I0);
    free(I1w);
    free(A);
    for (int i = 0; i < 14; i++)
        free(d[i]);
    free(It);
    free(Ixt);
    free(Iyt);
    free(a11);
    free(a12);
    free(a22);
    free(b1);
    free(b2);
}

int oref_dis_flow_refined(int32_t W, int32_t H, int32_t L, const float *pyr0,
                          const float *pyr1, int32_t ps, int32_t stride,
                          int32_t iters, double lambda,
                          const double *prev_flow, const oref_var_params *vr,
                          double *flow, double *patch_uv)
{
    if (L < 1 || L > 16 || ps < 1 || stride < 1 || iters < 0)
        return -1;
    int32_t lw[16], lh[16];
    size_t loff[16], poff[16];
    size_t off = 0, pofs = 0;
    int32_t w = W, h = H;
    for (int32_t l = 0; l < L; l++) {
        lw[l] = w;
        lh[l] = h;
        loff[l] = off;
        poff[l] = pofs;
        if (w < ps || h < ps)
            return -1;
        off += (size_t)w * h;
        pofs += (size_t)oref_patch_count(w, h, ps, stride);
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }

    double *Uc = NULL; /* dense flow of the coarser level, 2*Wc*Hc */
    for (int32_t l = L - 1; l >= 0; l--) {
        int32_t Wl = lw[l], Hl = lh[l];
        size_t np = (size_t)oref_patch_count(Wl, Hl, ps, stride);
        double *u0 = (double *)calloc(2 * np, sizeof(double));
        double *pu = (double *)malloc(sizeof(double) * 2 * np);
        /* start: zero (or the previous flow) at the coarsest level, the
         * coarser level's flow below it */
        if (l < L - 1)
            oref_patch_init_coarser(Wl, Hl, ps, stride, Uc, lw[l + 1], lh[l + 1], u0);
        else if (prev_flow)
            oref_patch_init_previous(Wl, Hl, l, ps, stride, prev_flow, W, H, u0);
        oref_dis_level(Wl, Hl, pyr0 + loff[l], pyr1 + loff[l], ps, stride,
                       iters, lambda, u0, pu);
        if (patch_uv)
            memcpy(patch_uv + 2 * poff[l], pu, sizeof(double) * 2 * np);
        double *Ul = (double *)malloc(sizeof(double) * 2 * (size_t)Wl * Hl);
        oref_densify(Wl, Hl, pyr0 + loff[l], pyr1 + loff[l], ps, stride, pu, Ul);
        if (vr)
            oref_var_refine(Wl, Hl, pyr0 + loff[l], pyr1 + loff[l], Ul, vr->outer,
                            vr->inner, vr->alpha, vr->gamma, vr->delta,
                            vr->omega);
        free(Uc);
        Uc = Ul;
        free(u0);
        free(pu);
    }
    memcpy(flow, Uc, sizeof(double) * 2 * (size_t)W * H);
    free(Uc);
    return 0;
}

int oref_dis_flow_warm(int32_t W, int32_t H, int32_t L, const float *pyr0,
                       const float *pyr1, int32_t ps, int32_t stride,
                       int32_t iters, double lambda, const double *prev_flow,
                       double *flow, double *patch_uv)
{
    return oref_dis_flow_refined(W, H, L, pyr0, pyr1, ps, stride, iters,
                                 lambda, prev_flow, NULL, flow, patch_uv);
}

int oref_dis_flow(int32_t W, int32_t H, int32_t L, const float *pyr0,
                  const float *pyr1, int32_t ps, int32_t stride,
                  int32_t iters, double lambda, double *flow,
                  double *patch_uv)
{
    return oref_dis_flow_warm(W, H, L, pyr0, pyr1, ps, stride, iters, lambda,
                              NULL, flow, patch_uv);
}

/* ------------------------------------------------------------------------ */
/* Section III-D names the paper's flow block: an update-prediction filter  */
/* that predicts the flow by image warping, carries it from one window to   */
/* the next (its memory effect) and stacks the loops over pyramid layers,   */
/* each layer with a regularisation weight and smoothing iterations          */
/* (Sec. IV-A).  The reading below is spelled out in the header.            */
/* ------------------------------------------------------------------------ */
/* bilinear interpolation of a double field, replicated border */
static double bilinear_d(const double *f, int32_t W, int32_t H, double sx,
                         double sy)
{
    double fx = floor(sx), fy = floor(sy);
    double ax = sx - fx, ay = sy - fy;
    if (fx < -2.0)
        fx = -2.0;
    if (fx > W + 2.0)
        fx = W + 2.0;
    if (fy < -2.0)
        fy = -2.0;
    if (fy > H + 2.0)
        fy = H + 2.0;
    int64_t x0 = (int64_t)fx, y0 = (int64_t)fy;
    double f00 = px_clamped(f, W, H, x0, y0);
    double f10 = px_clamped(f, W, H, x0 + 1, y0);
    double f01 = px_clamped(f, W, H, x0, y0 + 1);
    double f11 = px_clamped(f, W, H, x0 + 1, y0 + 1);
    return (1.0 - ay) * ((1.0 - ax) * f00 + ax * f10) +
           ay * ((1.0 - ax) * f01 + ax * f11);
}

void oref_ff_transport(int32_t W, int32_t H, const double *U, double *P)
{
    size_t N = (size_t)W * H;
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            size_t q = (size_t)y * W + x;
            double sx = x - U[q], sy = y - U[N + q];
            P[q] = bilinear_d(U, W, H, sx, sy);
            P[N + q] = bilinear_d(U + N, W, H, sx, sy);
        }
}

void oref_ff_smooth(int32_t W, int32_t H, int32_t iters, double *F)
{
    size_t N = (size_t)W * H;
    double *T = malloc(2 * N * sizeof(double));
    for (int32_t it = 0; it < iters; it++) {
        for (int c = 0; c < 2; c++) {
            const double *f = F + c * N;
            for (int32_t y = 0; y < H; y++)
                for (int32_t x = 0; x < W; x++)
                    T[c * N + (size_t)y * W + x] =
                        (px_clamped(f, W, H, x, y) + px_clamped(f, W, H, x - 1, y) +
                         px_clamped(f, W, H, x + 1, y) + px_clamped(f, W, H, x, y - 1) +
                         px_clamped(f, W, H, x, y + 1)) / 5.0;
        }
        memcpy(F, T, 2 * N * sizeof(double));
    }
    free(T);
}

int oref_flow_filter(int32_t W, int32_t H, int32_t L, const float *pyr0,
                     const float *pyr1, int32_t layers, const double *gamma,
                     const int32_t *smooth, double *state, double *flow)
{
    if (W < 1 || H < 1 || L < 1 || L > 64 || layers < 1 || layers > L)
        return -1;
    int32_t w[64], h[64];
    size_t off[64], soff[64];
    w[0] = W;
    h[0] = H;
    off[0] = soff[0] = 0;
    for (int32_t l = 1; l < L; l++) {
        w[l] = (w[l - 1] + 1) / 2;
        h[l] = (h[l - 1] + 1) / 2;
        off[l] = off[l - 1] + (size_t)w[l - 1] * h[l - 1];
        soff[l] = soff[l - 1] + 2 * (size_t)w[l - 1] * h[l - 1];
    }
    for (int32_t l = 0; l < layers; l++)
        if (gamma[l] <= 0.0 || smooth[l] < 0)
            return -1;
    double *Dc = NULL; /* the coarser layer's innovation */
    for (int32_t l = layers - 1; l >= 0; l--) {
        const int32_t Wl = w[l], Hl = h[l];
        const size_t N = (size_t)Wl * Hl;
        const float *I0 = pyr0 + off[l], *I1 = pyr1 + off[l];
        double *U = state + soff[l];
        double *Psi = malloc(2 * N * sizeof(double));
        double *Phi = malloc(2 * N * sizeof(double));
        oref_ff_transport(Wl, Hl, U, Psi);
        if (Dc) {
            const int32_t Wc = w[l + 1], Hc = h[l + 1];
            const size_t Nc = (size_t)Wc * Hc;
            for (int32_t y = 0; y < Hl; y++)
                for (int32_t x = 0; x < Wl; x++) {
                    int32_t X = x / 2, Y = y / 2;
                    if (X > Wc - 1)
                        X = Wc - 1;
                    if (Y > Hc - 1)
                        Y = Hc - 1;
                    size_t q = (size_t)y * Wl + x, qc = (size_t)Y * Wc + X;
                    Psi[q] += 2.0 * Dc[qc];
                    Psi[N + q] += 2.0 * Dc[Nc + qc];
                }
        }
        for (int32_t y = 0; y < Hl; y++)
            for (int32_t x = 0; x < Wl; x++) {
                size_t q = (size_t)y * Wl + x;
                double gx = 255.0 * 0.5 * (at_clamped(I0, Wl, Hl, x + 1, y) - at_clamped(I0, Wl, Hl, x - 1, y));
                double gy = 255.0 * 0.5 * (at_clamped(I0, Wl, Hl, x, y + 1) - at_clamped(I0, Wl, Hl, x, y - 1));
                double r = 255.0 * (bilinear(I1, Wl, Hl, x + Psi[q], y + Psi[N + q]) - (double)I0[q]);
                double k = r / (gx * gx + gy * gy + gamma[l]);
                Phi[q] = Psi[q] - gx * k;
                Phi[N + q] = Psi[N + q] - gy * k;
            }
        oref_ff_smooth(Wl, Hl, smooth[l], Phi);
        for (size_t q = 0; q < 2 * N; q++) {
            U[q] = Phi[q];
            Phi[q] -= Psi[q]; /* the innovation, for the finer layer */
        }
        free(Psi);
        free(Dc);
        Dc = Phi;
    }
    free(Dc);
    memcpy(flow, state, 2 * (size_t)W * H * sizeof(double));
    return 0;
}
