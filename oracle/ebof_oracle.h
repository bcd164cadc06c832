/*
 * ebof_oracle.h -- plain CPU oracle of the event-based optical-flow hot path
 * (Brebion, Moreau, Davoine, "Real-Time Optical Flow for Vehicular Perception
 * with Low- and High-Resolution Event Cameras", arXiv 2112.10591).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or helper with the GPU
 * library and includes none of its files.
 *
 * Conventions shared with the GPU library only through the documented data
 * layout (not through code):
 *   - images are row-major, pitch = width, pixel (x, y) at index y*W + x;
 *   - a pyramid of L levels stores level 0 first, then level 1, ... each
 *     tightly packed; level l+1 has size ((W_l+1)/2, (H_l+1)/2);
 *   - the squared distance of a pixel in an image with no edge pixel at all is
 *     INT32_MAX;
 *   - flows are two planes (u then v), u along +x (right), v along +y (down).
 *
 * Floating point: every intermediate is double precision.  Values that the
 * method stores as FP32 (the distance surface and its pyramid levels) are
 * rounded to float once, from the double result.
 */
#ifndef EBOF_ORACLE_H
#define EBOF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Section III-A: binary edge image of the events with t0 <= t < t0 + dt.
 * Polarity is not an input (the paper ignores it).  Events outside the
 * window or outside the W x H sensor are not binned.  E gets W*H bytes of
 * 0/1.  Returns the number of events not binned. */
int64_t oref_edge_image(int32_t W, int32_t H, const uint16_t *x,
                        const uint16_t *y, const int64_t *t, int64_t n,
                        int64_t t0, int64_t dt, uint8_t *E);

/* Algorithm 1 (denoising): an edge pixel with fewer than n_d edge pixels
 * among its 4 direct neighbours in E stops being an edge.  Reads E only. */
void oref_denoise(int32_t W, int32_t H, const uint8_t *E, int32_t n_d,
                  uint8_t *Ed);

/* Algorithm 2 (filling): a non-edge pixel with at least n_f edge pixels
 * among its 4 direct neighbours in Ed becomes an edge.  Reads Ed only. */
void oref_fill(int32_t W, int32_t H, const uint8_t *Ed, int32_t n_f,
               uint8_t *Edf);

/* Squared Euclidean distance to the closest edge pixel (the d_Euc of
 * equation (1), squared), by its definition: a minimum over all edge pixels.
 * O(W*H*#edges); for small images and for sampled pixels. */
void oref_edt_brute(int32_t W, int32_t H, const uint8_t *E, int32_t *D2);
int32_t oref_edt_brute_at(int32_t W, int32_t H, const uint8_t *E, int32_t px,
                          int32_t py);

/* The same quantity by the exact separable method (column distances, then a
 * lower envelope of parabolas per row), the family of algorithms Section
 * III-C names for its implementation. */
void oref_edt_separable(int32_t W, int32_t H, const uint8_t *E, int32_t *D2);

/* Equation (1): S = 1 - exp(-sqrt(D2) / alpha), rounded once to float. */
void oref_surface(int64_t n, const int32_t *D2, double alpha, float *S);

/* The distance-surface alternatives of the ablation study (Sec. IV-B), from
 * the squared distance D2 with d = sqrt(D2), each rounded once to float:
 *   kind 0, eq. (1):       1 - exp(-d / alpha)
 *   kind 1, DS_L:          d
 *   kind 2, DS_LB:         min(d, d_sat) with d_sat = alpha ln 255 (eq. 3)
 *   kind 3, DS_Log:        ln(d + 1)
 * The no-edge sentinel D2 = INT32_MAX goes through the same formula. */
void oref_surface_kind(int64_t n, const int32_t *D2, double alpha, int32_t kind,
                       float *S);

/* Sec. IV, evaluation metrics, of flow u against ground truth v (both two
 * planes of n values) over the pixels where mask != 0 (every pixel when mask
 * is NULL): *aee = mean |v - u| (Euclidean), *outliers = fraction of those
 * pixels with |v - u| > 3 px and > 5 % of |v|.  Returns the number of pixels
 * counted (0: both outputs 0). */
int64_t oref_flow_errors(int64_t n, const double *u, const double *v,
                         const uint8_t *mask, double *aee, double *outliers);

/* Sec. IV, flow warp loss.  The events of one window (t0 <= t < t0 + dt, on
 * the W x H sensor) are accumulated into two images: at their own pixel
 * (uncompensated), and moved back to the window start by the flow at their
 * pixel scaled by their time in the window, x' = x - u(x, y) (t - t0) / dt
 * (likewise y), voting bilinearly into the four pixels around x' (votes off
 * the sensor are lost).  Each event votes its polarity (+1 / -1) when pol is
 * given, else 1.  flow: two planes of W*H doubles, pixels per dt.
 * var_comp / var_uncomp get the variances of the two images over all W*H
 * pixels; returns var_comp / var_uncomp (0 when var_uncomp is 0). */
double oref_fwl(int32_t W, int32_t H, const uint16_t *x, const uint16_t *y,
                const int64_t *t, const int8_t *pol, int64_t n, int64_t t0,
                int64_t dt, const double *flow, double *var_comp,
                double *var_uncomp);

/* Adaptive windows (the adaptive accumulation time the Conclusion proposes,
 * with the area event count as the rule): scanning a time-ordered stream from
 * event i0, each on-sensor event counts for its square of the area x area
 * tiling from (0, 0); returns one past the event that brings some square to
 * k_events, or n when none does. */
int64_t oref_window_end_area(int32_t W, int32_t H, const uint16_t *x,
                             const uint16_t *y, int64_t n, int64_t i0,
                             int32_t area, int32_t k_events);

/* One pyramid reduction: out(X,Y) = sum_{i,j=-2..2} k_i k_j in(2X+i, 2Y+j),
 * k = [1 4 6 4 1]/16, reflect-101 border.  out is ((W+1)/2) x ((H+1)/2). */
void oref_pyr_down(int32_t W, int32_t H, const float *in, float *out);

/* Dense inverse search flow from pyramid pyr0 (reference, window k-1) to
 * pyramid pyr1 (window k), both L levels in the packed layout above.
 * flow gets 2*W*H doubles (u plane, v plane) at level 0.  patch_uv, when not
 * NULL, gets the final patch displacements of every level, level 0 first,
 * patches row-major, (u, v) interleaved.  Returns 0, or -1 on bad arguments
 * (a level smaller than the patch, ps < 1, stride < 1, iters < 0). */
int oref_dis_flow(int32_t W, int32_t H, int32_t L, const float *pyr0,
                  const float *pyr1, int32_t ps, int32_t stride,
                  int32_t iters, double lambda, double *flow,
                  double *patch_uv);

/* The same with a warm start: when prev_flow (2*W*H doubles, the dense
 * level-0 flow of the previous window pair) is not NULL, the coarsest level
 * starts from it (oref_patch_init_previous) instead of from zero. */
int oref_dis_flow_warm(int32_t W, int32_t H, int32_t L, const float *pyr0,
                       const float *pyr1, int32_t ps, int32_t stride,
                       int32_t iters, double lambda, const double *prev_flow,
                       double *flow, double *patch_uv);

/* The steps of one level, as oref_dis_flow composes them.  Patch
 * displacements u0 / pu are (u, v) interleaved, patches row-major; a flow
 * U is two planes of doubles.
 *   oref_patch_init_coarser: u0 of a W x H level from the coarser level's
 *     dense flow Uc (Wc x Hc): twice Uc at (floor((o+ps/2)/2)) per axis,
 *     clamped into the coarser image.
 *   oref_patch_init_previous: u0 of level `level` (W x H) of a W0 x H0
 *     sensor from a dense level-0 flow Up: Up at ((o+ps/2) << level) per
 *     axis, clamped into the sensor, divided by 2^level.
 *   oref_dis_level: the inverse search of every patch from u0 (NULL = 0)
 *     into pu, with the outlier reset.
 *   oref_densify: the weighted mean of the covering patches' displacements
 *     into U (2*W*H). */
void oref_patch_init_coarser(int32_t W, int32_t H, int32_t ps, int32_t stride,
                             const double *Uc, int32_t Wc, int32_t Hc,
                             double *u0);
void oref_patch_init_previous(int32_t W, int32_t H, int32_t level, int32_t ps,
                              int32_t stride, const double *Up, int32_t W0,
                              int32_t H0, double *u0);
void oref_dis_level(int32_t W, int32_t H, const float *I0, const float *I1,
                    int32_t ps, int32_t stride, int32_t iters, double lambda,
                    const double *u0, double *pu);
void oref_densify(int32_t W, int32_t H, const float *I0, const float *I1,
                  int32_t ps, int32_t stride, const double *pu, double *U);

/* Variational refinement (the third stage of dense inverse search) of a
 * dense flow U (2*W*H doubles, in/out) between I0 and I1 (W x H floats, the
 * [0,1] surfaces taken on the 8-bit scale, x255): `outer` fixed-point
 * iterations, each weighting the linearised brightness-constancy residual
 * It + Ix du + Iy dv (weight delta), the gradient-constancy residuals
 * Ixt + Ixx du + Ixy dv and Iyt + Ixy du + Iyy dv (weight gamma) and the
 * smoothness of the refined flow (weight alpha) by the robust penalty's
 * derivative 1 / sqrt(s^2 + 1e-6) at the current increment, then `inner`
 * red-black block SOR sweeps (relaxation omega) on the 2x2 systems of the
 * increment; finally U += (du, dv).  Derivatives: central differences with
 * replicated border, Ix, Iy, Ixx, Iyy, Ixy (symmetrised) of the average of
 * I0 and the warped I1(x + U) (bilinear, replicated border), It = I1w - I0,
 * Ixt, Iyt = the warped image's gradient minus the reference's. */
typedef struct {
    int32_t outer, inner;
    double alpha, gamma, delta, omega;
} oref_var_params;
void oref_var_refine(int32_t W, int32_t H, const float *I0, const float *I1,
                     double *U, int32_t outer, int32_t inner, double alpha,
                     double gamma, double delta, double omega);

/* oref_dis_flow_warm with the refinement applied to each level's dense flow
 * before it starts the next level (vr NULL: no refinement). */
int oref_dis_flow_refined(int32_t W, int32_t H, int32_t L, const float *pyr0,
                          const float *pyr1, int32_t ps, int32_t stride,
                          int32_t iters, double lambda,
                          const double *prev_flow, const oref_var_params *vr,
                          double *flow, double *patch_uv);

/* Update-prediction flow filter: the kind of frame-based flow block the
 * paper's Sec. III-D selects (a predictive filter: the flow is predicted by
 * warping and propagated in time, with update-prediction loops stacked over
 * pyramid layers, each with its own regularisation weight and number of
 * smoothing iterations, the Sec. IV-A parameters).  The paper gives no
 * equations; this reading is the one the GPU library implements:
 *   state: per layer l < layers (pyramid level l, W_l x H_l), the flow U_l of
 *     the previous window pair (pixels of that level per window), two planes;
 *     zero before the first pair.
 *   for l = layers-1 down to 0:
 *     prediction  P_l(x) = U_l(x - U_l(x)): the previous flow carried along
 *                 itself over one window (bilinear, replicated border);
 *                 Psi_l = P_l, plus, below the top layer, twice the coarser
 *                 layer's innovation D_{l+1} at the parent pixel
 *                 (floor(x/2), floor(y/2));
 *     update      with g = 255 grad I0(x) (central differences, replicated
 *                 border) and r = 255 (I1(x + Psi_l(x)) - I0(x)) (bilinear,
 *                 replicated border): Phi = Psi_l - g r / (|g|^2 + gamma_l),
 *                 the minimiser of (g.(Phi - Psi_l) + r)^2 +
 *                 gamma_l |Phi - Psi_l|^2;
 *     smoothing   smooth_l Jacobi iterations Phi <- mean of Phi at x and its
 *                 four neighbours (replicated border), both planes;
 *     U_l <- Phi, D_l = Phi - Psi_l.
 *   The output flow is U_0.
 * oref_ff_transport: P from U (one W x H layer, two planes each).
 * oref_ff_smooth: `iters` iterations on F (two planes, in place).
 * oref_flow_filter: pyr0 / pyr1 of L >= layers levels in the packed layout;
 *   state: 2 * sum_{l<layers} W_l H_l doubles, layer 0 first (in/out);
 *   flow: 2*W*H doubles (U_0).  Returns 0, or -1 on bad arguments. */
void oref_ff_transport(int32_t W, int32_t H, const double *U, double *P);
void oref_ff_smooth(int32_t W, int32_t H, int32_t iters, double *F);
int oref_flow_filter(int32_t W, int32_t H, int32_t L, const float *pyr0,
                     const float *pyr1, int32_t layers, const double *gamma,
                     const int32_t *smooth, double *state, double *flow);

/* Number of patches of one level: ceil((W-ps)/stride)+1 by the same in y. */
int64_t oref_patch_count(int32_t W, int32_t H, int32_t ps, int32_t stride);

#ifdef __cplusplus
}
#endif

#endif /* EBOF_ORACLE_H */
