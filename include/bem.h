/*
 * bem.h - C ABI of the MI355X (gfx950) differential-BEM hot path for fitting
 * diffusion curves to noisy Monte Carlo samples.
 *
 * The method: colours u(x) in the unit-square image domain solve Laplace's
 * equation away from handle curves, with prescribed jumps of the colour (wd)
 * and of its normal derivative (wc) across each handle and zero Neumann data
 * on the outer boundary (paper Sec. 2.1, Eq. laplace / Eq. neumann; Sec. 3.1.1,
 * Eq. bie / Eq. handleterm).  The outer boundary is discretised into constant
 * elements and solved once by a Galerkin system (Eq. bie_galerkin) whose
 * one-dimensional null space is removed by dropping the smallest singular
 * value (Sec. 3.1.3); derivatives with respect to handle parameters solve the
 * same system with differentiated right-hand sides (Eq. diffbie, Sec. 3.2);
 * a Levenberg-Marquardt step uses Monte Carlo estimates of J^T J and J^T r
 * (Eq. optimstep, Eq. losshessian, Eq. lossjacobian, Sec. 4.3).
 *
 * Conventions shared by every entry point
 *  - Handles (bem_opts.handle_model), each cut at t = k/S into S straight
 *    segments (K = H*S); theta is [H,Q] float64 row-major, P = Q*H parameters,
 *    and every Jacobian/gradient uses theta's column order.
 *    BEM_HANDLE_CUBIC (Q = 20): cubic Bezier curves, per handle
 *      [P0x P0y P1x P1y P2x P2y P3x P3y | wd0 RGB | wd1 RGB | wc0 RGB | wc1 RGB]
 *    where wd/wc at end 0 (t=0) and end 1 (t=1) are interpolated linearly in t.
 *    BEM_HANDLE_STRAIGHT (Q = 10): the paper's own handles (Sec. 3.2 line
 *    segments; Sec. 4.1 two end points, jumps constant over the handle),
 *      [Ax Ay Bx By | wd RGB | wc RGB],
 *    the segment A -> B with vertices A + (k/S)(B - A).  S = 1 is exact: the
 *    closed-form integrals of a straight piece with constant density do not
 *    change under subdivision.
 *  - Orientation: a segment a->b has right normal n = (tau_y, -tau_x); wd is
 *    the colour on the left minus the colour on the right, wc the jump of the
 *    derivative along n.  The outer boundary is counter-clockwise, so n is
 *    outward there.
 *  - The handle kernels are regularised r^2 -> r^2 + eps^2 (Sec. 3.1.3); the
 *    outer-boundary kernels are exact.
 *  - Samples x are [N,2] float64 strictly inside the subdomain: the open unit
 *    square for bem_build, the region the elements bound for bem_build_elements.
 *  - All array pointers are DEVICE pointers owned by the caller unless marked
 *    (host).  The library owns only the context and its internal workspaces,
 *    which it grows with hipMalloc on first use of a size and frees in
 *    bem_destroy.
 *  - Calls enqueue on `stream` and return without a host synchronisation,
 *    except where stated (lm_step; growth of a workspace; the first bem_jtj
 *    of a context for a given H, which uploads its Gram work list).
 *  - Every call returns a bem_status; nothing throws across the ABI.  On an
 *    error, outputs are unspecified and bem_last_error() describes it.
 *  - A context is not thread-safe; use one context per stream.
 */
#ifndef BEM_H
#define BEM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bem_ctx bem_ctx;

typedef enum {
    BEM_OK = 0,
    BEM_EINVAL = -1,     /* bad argument (null pointer, size out of range, bad enum)       */
    BEM_ENOMEM = -2,     /* device allocation failed                                      */
    BEM_ESTATE = -3,     /* call order: the boundary system is not built/factored yet     */
    BEM_ENOTPD = -4,     /* Cholesky of the damped normal matrix met a non-positive pivot */
    BEM_EHIP = -5,       /* a HIP runtime call or kernel launch failed                    */
    BEM_ENUMERIC = -6    /* non-finite value where a finite one is required               */
} bem_status;

/* Arithmetic of the sample x segment sweeps.
 * FP64 : every pair in float64; u and cotangents are float64.
 * MIXED: pairs in float32 except near-singular pairs (both segment end points
 *        within max(2 nf, nf + 1)*L of the sample, nf = near_factor, which
 *        contains every sample closer than nf*L to the segment), which are
 *        evaluated in
 *        float64 from the float64 inputs; u and cotangents are float32; every
 *        reduction over samples is finished in float64.  The float64 sums of
 *        near pairs in bem_eval and bem_vjp are accumulated with atomics, so
 *        MIXED results can differ in their last bits from call to call; FP64
 *        results are reproducible.  The boundary matrix, its factorisation and
 *        solves and the LM solve are float64 in both modes; the boundary
 *        right-hand side (the handles' field at the elements' Gauss points)
 *        takes the same float32 / float64 split as the sweeps in MIXED.
 *        Near pairs go to a list with a per-context capacity per 64 samples
 *        (1024 at first, at most 16384 and 4 GiB of list); the samples whose
 *        pairs do not fit are evaluated by a slower sweep that handles their
 *        near pairs inline, with the same result to rounding.  lm_step raises
 *        the capacity when its sweeps overflow (a workspace for later calls of
 *        the context too); the other calls keep the capacity reached. */
typedef enum { BEM_PREC_FP64 = 0, BEM_PREC_MIXED = 1 } bem_prec;

/* Arithmetic of the Gram contraction that forms J^T J and J^T r.
 * FP64         : float64 tiles, float64 products and accumulation on float64
 *                MFMA (v_mfma_f64_16x16x4f64).
 * FP32_MFMA    : float32 J tiles, float32 MFMA, float32 accumulation within
 *                a sample tile, float64 across tiles.
 * BF16X3_MFMA  : J split as hi + lo bfloat16, hi*hi + hi*lo + lo*hi on bf16
 *                MFMA with float32 accumulation within a third of a sample
 *                tile, float64 across thirds and tiles (fixed order).
 * FP64_VALU    : as FP64, with the products on the float64 vector ALUs.
 * Every float64 product of the library (the Gram's contraction to J^T J, the
 * boundary derivatives Z = A+ dF/dtheta) runs on float64 MFMA in all modes. */
typedef enum { BEM_GRAM_FP64 = 0, BEM_GRAM_FP32_MFMA = 1, BEM_GRAM_BF16X3_MFMA = 2, BEM_GRAM_FP64_VALU = 3 } bem_gram;

/* Handle parametrisation (see the conventions above). */
typedef enum { BEM_HANDLE_CUBIC = 0, BEM_HANDLE_STRAIGHT = 1 } bem_handle_model;

typedef struct {
    int32_t elems_per_side;   /* outer elements per side of the unit square (256: length 1/256, Sec. 3.1.3) */
    int32_t segs_per_handle;  /* S >= 1 */
    double eps;               /* handle-kernel regularisation (1e-2 in the paper's experiments); >= 0 */
    double near_factor;       /* MIXED near-pair threshold in segment lengths (1.0); > 0 */
    int32_t tile_rows;        /* sample rows per J tile in bem_jtj (0: automatic) */
    int32_t device;           /* HIP device ordinal the context lives on */
    int32_t handle_model;     /* bem_handle_model: Q = 20 (cubic) or 10 (straight) parameters per handle */
} bem_opts;

/* Host-side state of the LM iteration (Sec. 4.3).  lambda is the damping
 * factor; the mean colour cbar is either the running mean of every target
 * seen (mean_rule 0: the paper's rule, outside LM) or the least-squares
 * constant mean(T - u_bem) of the current step (mean_rule 1). */
typedef struct {
    double lambda;            /* in/out: damping (clamped to [1e-12, 1e12])         */
    double cbar[3];           /* out: mean colour used in this step                 */
    double cbar_sum[3];       /* in/out: running sum of targets (mean_rule 0)       */
    int64_t cbar_count;       /* in/out: number of target rows summed               */
    int32_t mean_rule;        /* in: 0 running mean of targets, 1 least squares     */
    int32_t accepted;         /* out: 1 if the step lowered the loss                */
    double loss_before;       /* out: (1/2N) sum |u - T|^2 at theta                 */
    double loss_after;        /* out: same at the trial parameters                  */
    int32_t chol_retries;     /* out: extra damping rounds after a failed Cholesky  */
    int32_t compat;           /* in: 1 enforces the compatibility condition          */
    double compat_violation;  /* out: max_c |a_c . theta'| / sum |a_c theta'| (compat) */
    double reg_value;         /* out: regularisation terms at theta (in loss_before)  */
    int32_t snap_pairs;       /* out: end point pairs snapped in this step            */
    int64_t data_count;       /* in: M_H, samples drawn over the whole image, which
                                 divides the data terms (0: the step's own N; else >= N) */
} bem_lm_state;

/* Regularisation terms of the LM step (Sec. 4.4).  Each enters the step with its
 * analytic gradient and Hessian, added to the normal equations (g and H of
 * lm_step), and with its value added to the loss on both sides of the accept
 * test.  A weight of 0 switches a term off; all are off until
 * bem_set_regularization.  End points E0, E1 of a handle: straight A, B; cubic
 * P0, P3.  Jump vectors w: straight wd, wc; cubic wd0, wd1, wc0, wc1 (RGB).
 *   length    length_weight (l - length_max)^2 for each handle with
 *             l = |E1 - E0| > length_max;
 *   snapping  snap_weight |e - e'|^2 for each pair of end points e, e' of two
 *             different handles, closer than snap_dist, each of which has the
 *             other as its lowest snapping score
 *               snap_mix |e - e'| / snap_dist + (1 - snap_mix)(1 - |tau . tau'|)
 *             (tau: unit direction E1 - E0 of each handle, 0 for a zero-length
 *             handle; ties go to the lower end point index 2h + j).  The pairs
 *             are chosen at the step's theta and kept for its trial point;
 *   sparsity  lambda t tanh(sqrt(w . w + eps^2) / t) per jump vector, lambda =
 *             sparse_wd for wd and sparse_wc for wc.
 * The length and snapping Hessians are exact (positive semi-definite); the
 * sparsity term's curvature along w is negative (the term saturates) and is
 * left out, so that the approximate Hessian stays positive definite for the
 * Cholesky solve (Sec. 4.3): it contributes f'(s)/s (I - w w^T / s^2),
 * s = sqrt(w . w + eps^2). */
typedef struct {
    double length_weight;     /* >= 0 */
    double length_max;        /* >= 0 */
    double snap_weight;       /* >= 0 */
    double snap_dist;         /* > 0 when snap_weight > 0 */
    double snap_mix;          /* in [0, 1] */
    double sparse_wd;         /* >= 0 */
    double sparse_wc;         /* >= 0 */
    double sparse_t;          /* > 0 when a sparsity weight is > 0 */
    double sparse_eps;        /* >= 0 */
} bem_reg;

/* Build the outer boundary (unit square, counter-clockwise, elems_per_side
 * equal elements per side, M = 4*elems_per_side) and assemble the float64
 * Galerkin matrix A of Eq. bie_galerkin: A_ii = |G_i|/2, A_ij = 3x3-point
 * Gauss integral of dG/dn_y over G_i x G_j, the coincident term zero
 * (Sec. 3.1.3).  *out receives a new context (host).  opts is host memory,
 * copied.  Errors: EINVAL (null pointer, elems_per_side < 2 or > 1024,
 * S < 1 or > 1024, eps < 0 or not finite, near_factor <= 0, bad
 * handle_model), ENOMEM, EHIP. */
int bem_build(const bem_opts* opts, hipStream_t stream, bem_ctx** out);

/* The same for an outer boundary made of any M straight elements (Sec. 4.1: each
 * subdomain has its own boundary, which may be non-convex, open or
 * self-intersecting).  elems (host, copied) is [M,4] float64 row-major, element i
 * running from (elems[4i], elems[4i+1]) to (elems[4i+2], elems[4i+3]); a closed
 * boundary runs counter-clockwise, so that the right normal points out of the
 * subdomain.  The Galerkin matrix, its truncated-SVD solve (which drops the
 * smallest singular value whether or not the boundary is closed) and every later
 * call are those of bem_build with these elements; opts.elems_per_side is
 * ignored.  Elements must not overlap one another.  Samples of the later calls
 * are the subdomain's.  Errors: as bem_build, EINVAL (null elems, M not in
 * [2, 4096], a zero-length or non-finite element). */
int bem_build_elements(const bem_opts* opts, const double* elems, int32_t M, hipStream_t stream,
                       bem_ctx** out);

/* One-time float64 factorisation (Sec. 3.1.3, factor once and reuse, Sec. 4.2):
 * the smallest singular triplet (sigma_n, u_n, v_n) of A by inverse iteration
 * with a pivoted LU of A, the deflated matrix B = A + (s - sigma_n) u_n v_n^T
 * (s = |A|_F / sqrt(M)), and the explicit truncated pseudo-inverse
 * A+ = B^{-1} - v_n u_n^T / s, which equals the SVD solve that drops the
 * smallest singular value.  Synchronises the stream.
 * Errors: ESTATE (not built), ENUMERIC (zero pivot), ENOMEM, EHIP. */
int bem_factor(bem_ctx* ctx, hipStream_t stream);

/* Forward evaluation u(x) = cbar + sum_j beta_j(x) U_j + f(x) (Eq. bie with
 * alpha = 1 plus the mean colour, Sec. 3.1.3), where f is the handle term of
 * Eq. handleterm, U = A+ F the solved outer-boundary values with
 * F_i = int_{G_i} f by 3-point Gauss, and beta_j(x) = -int_{G_j} dG/dn_y.
 * theta [H,Q] f64, x [N,2] f64, cbar[3] (host), u [N,3] row-major, float64
 * for FP64 and float32 for MIXED.  H = 0 or N = 0 are allowed.
 * Errors: ESTATE (not factored), EINVAL, ENOMEM, EHIP. */
int bem_eval(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N,
             const double* cbar, void* u, bem_prec prec, hipStream_t stream);

/* Vector-Jacobian product: grad[p] = sum_x sum_c gbar_c(x) du_c(x)/dtheta_p,
 * the reverse-mode form of the differential BIE (Eq. diffbie): segment
 * adjoints over all samples, psi = sum_x gbar(x) beta(x), mu = A+^T psi, and
 * the segment adjoints at the boundary Gauss points with cotangent mu.
 * gbar [N,3] row-major (float64 for FP64, float32 for MIXED), grad [H,Q]
 * float64, overwritten.  The mean colour does not depend on theta.
 * MIXED with N >= 65,536 samples: a copy of x and gbar reordered cell by cell
 * (a 32 x 32 grid of Morton-ordered cells over the outer boundary's bounding
 * box; 80 bytes per sample of context workspace) is processed, so that the
 * near pairs of a wavefront form long runs; the result depends on the order
 * only through rounding.
 * Errors: as bem_eval. */
int bem_vjp(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N,
            const void* gbar, double* grad, bem_prec prec, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): bem_vjp in FP64 that
 * calls no hipMalloc / hipFree and no allocating library routine.  Same
 * arguments and result as bem_vjp(..., BEM_PREC_FP64, ...) (gbar float64), to
 * rounding: every workspace of the call (segment and element tables, partial
 * sums, psi, mu, the boundary Gauss points) is carved from a static 64 MiB
 * device array of the library, one per device, held until the process ends
 * (its address is looked up once per device on the first call there).  The
 * context must be built and factored (those calls allocate).  Sizes whose
 * workspace exceeds the array fail with BEM_EINVAL and a message: with
 * M = 1024 outer elements every K = H*S <= 13,376 segments fits for any N
 * (the LM workload's 8,192 take 53.5 MiB); nothing needs to start at zero.  Every call on a device shares that device's array, so calls that
 * overlap on one device (two streams, two threads, two contexts) race: the
 * caller must serialise them.  No profiling events are recorded for the call.
 * Errors: as bem_vjp. */
int bem_vjp_noalloc(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N,
                    const double* gbar, double* grad, hipStream_t stream);

/* Monte Carlo normal equations with uniform samples (p = 1 on the unit
 * square; Eq. losshessian, Eq. lossjacobian):
 *   JtJ = (1/N) sum_x sum_c J_c(x)^T J_c(x)   [P,P] float64 (full, symmetric)
 *   Jtr = (1/N) sum_x sum_c J_c(x)^T r_c(x)   [P]   float64
 * with J_c(x) = du_c(x)/dtheta.  resid [N,3] (float64 for FP64, float32 for
 * MIXED).  The Gram contraction runs in `gram` arithmetic.  The Gram's work
 * list is uploaded (with a host synchronisation) on the first call for a given
 * H, handle model and `gram` and kept on the device; later calls only enqueue.
 * Errors: as bem_eval. */
int bem_jtj(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N,
            const void* resid, double* JtJ, double* Jtr, bem_gram gram, bem_prec prec,
            hipStream_t stream);

/* One Levenberg-Marquardt step (Eq. optimstep, Sec. 4.3) on the samples x
 * with targets T [N,3] float64, m = state->data_count (0: m = N):
 *   cbar update (state->mean_rule), u = u(theta), r = u - T, loss L0 = (1/2m) sum r^2,
 *   g = (1/m) sum J^T r by the adjoint (bem_vjp), H = (1/m) sum J^T J (bem_jtj's
 *   Gram; J^T r itself is not formed again),
 *   delta = (lambda diag(H) + H)^{-1} g by float64 Cholesky,
 *   theta' = theta - delta, L1 = loss at theta' on the same samples with cbar fixed;
 *   accept iff L1 < L0: theta <- theta', lambda /= 10; else lambda *= 10.
 * With state->compat = 1 the compatibility condition of Sec. 3.1.2 (zero net
 * flux of the normal-derivative jump, int over the handles of w_c = 0 per
 * channel, linear in the wc parameters for fixed end points: a_c . theta = 0)
 * is enforced as in Sec. 4.3: delta is the damped step restricted to
 * a_c . delta = 0 (a_c at the current end points; KKT system through its 3x3
 * Schur complement, 3 more Cholesky solves), and after the update the wc
 * parameters are projected orthogonally onto a_c . theta' = 0 with a_c at the
 * new end points; state->compat_violation reports what remains (rounding).
 * With regularisation terms set (bem_set_regularization) their gradient and
 * Hessian are added to g and H, and their value to L0 and L1 (snapping pairs
 * chosen at theta); state->reg_value and state->snap_pairs report them.
 * The data terms are Monte Carlo estimates over the m samples drawn for the
 * whole image (Eq. losshessian, Eq. lossjacobian divide by M_H): the step of one
 * subdomain (Sec. 4.3, block-diagonal Hessian) sums its own N samples and sets
 * data_count to the image's total, so that its data terms keep their weight
 * against the regularisation terms.
 * MIXED: the step works on a copy of x and target reordered cell by cell (a
 * 32 x 32 grid of Morton-ordered cells over the outer boundary's bounding box),
 * so that neighbouring samples share wavefronts; x and target themselves are
 * not modified, and the result depends on the order only through rounding.
 * If the near-pair list of the sweep at theta overflows, its capacity is raised
 * (to 1.25 times the largest wavefront count, rounded up to 256) and the sweep
 * repeated before the adjoint and the normal equations.
 * If the Cholesky fails, lambda is multiplied by 10 and the solve retried (at
 * most 10 times) before ENOTPD.  theta [H,Q] (device) is updated in place;
 * state (host) is read and written.  Synchronises the stream.
 * Errors: as bem_eval, EINVAL (data_count < 0 or 0 < data_count < N), ENOTPD,
 * ENUMERIC (non-finite loss or step). */
int lm_step(bem_ctx* ctx, double* theta, int32_t H, const double* x, int64_t N,
            const double* target, bem_lm_state* state, bem_gram gram, bem_prec prec,
            hipStream_t stream);

/* Set the regularisation terms lm_step adds (host struct, copied; NULL switches
 * every term off).  Errors: EINVAL (null context, a negative or non-finite
 * weight, snap_dist <= 0 or snap_mix outside [0, 1] with snapping on,
 * sparse_t <= 0 or sparse_eps < 0 with sparsity on). */
int bem_set_regularization(bem_ctx* ctx, const bem_reg* reg);

/* The regularisation terms set on the context at theta [H,Q] (device): *value
 * (host) = their sum, grad [P] and hess [P,P] (device, row-major, overwritten;
 * both NULL for the value only), *pairs (host, may be NULL) = the number of
 * snapped end point pairs.  Snapping compares every pair of end points
 * (O(H^2)) and is limited to H <= 65536.  Synchronises the stream.
 * Errors: ESTATE, EINVAL (one of grad / hess NULL, H out of range), ENOMEM, EHIP. */
int bem_regularization(bem_ctx* ctx, const double* theta, int32_t H, double* value, double* grad,
                       double* hess, int32_t* pairs, hipStream_t stream);

/* Handle pruning (Sec. 4.4, with the sparsity term): removes, in place, every
 * handle whose wd norm and wc norm (for cubic handles the larger over the two
 * ends) are both below threshold (a NaN norm counts as below), keeping the
 * order of the others in theta[0 : *H_out].  Rows past *H_out are unspecified.
 * Synchronises the stream.  Errors: ESTATE, EINVAL (threshold < 0 or not
 * finite, null H_out), ENOMEM, EHIP. */
int bem_prune(bem_ctx* ctx, double* theta, int32_t H, double threshold, int32_t* H_out, hipStream_t stream);

/* Samples grouped by subdomain (Sec. 4.1: each sample belongs to the subdomain its
 * camera ray hits first; Sec. 4.3: each subdomain's normal equations use its own
 * samples and are solved separately): a stable partition of x [N,2] and T [N,3]
 * (float64, device; T may be NULL) by labels [N] (int32, device) into x_out and
 * T_out (device, [N,2] / [N,3] rows reserved), so that the samples with label d
 * occupy rows offsets[d] .. offsets[d+1]-1 in their original order; labels
 * outside [0, D) are dropped (offsets[D] = rows kept).  offsets is host [D+1].
 * The workspace is ctx's (any context of the device).  Synchronises the stream.
 * Errors: EINVAL (null pointers, D not in [1, 1024], N < 0), ENOMEM, EHIP. */
int bem_partition_samples(bem_ctx* ctx, const int32_t* labels, int64_t N, int32_t D, const double* x,
                          const double* T, double* x_out, double* T_out, int64_t* offsets,
                          hipStream_t stream);

/* Explicit float64 Jacobian J [N,3,P] (row = sample*3 + channel), the
 * quantity the paper differentiates in Sec. 3.2.  For tests and small N.
 * Errors: as bem_eval. */
int bem_jacobian(bem_ctx* ctx, const double* theta, int32_t H, const double* x, int64_t N,
                 double* J, hipStream_t stream);

/* Intermediate quantities of the forward path, float64, for inspection:
 * F [M,3] = int_{G_i} f (right-hand side of Eq. bie_galerkin) and
 * U [M,3] = A+ F.  Either pointer may be NULL.  Errors: as bem_eval. */
int bem_boundary_solve(bem_ctx* ctx, const double* theta, int32_t H, double* F, double* U,
                       hipStream_t stream);

/* Copy the assembled matrix A [M,M] (after bem_build) or the truncated
 * pseudo-inverse A+ [M,M] (after bem_factor), row-major float64, into a
 * caller buffer; which = 0 for A, 1 for A+.  Errors: ESTATE, EINVAL, EHIP. */
int bem_get_matrix(bem_ctx* ctx, int32_t which, double* out, hipStream_t stream);

/* Number of outer elements M (host); 0 for a null context. */
int32_t bem_num_elements(const bem_ctx* ctx);

/* Near-pair list capacity of the MIXED sweeps in slots per 64 samples (the
 * description of bem_prec says how it grows); 0 for a null context. */
int32_t bem_near_capacity(const bem_ctx* ctx);

/* Smallest singular value sigma_n and the deflation shift s found by bem_factor (host). */
int bem_factor_info(const bem_ctx* ctx, double* sigma_n, double* shift);

/* Kernel timing with HIP events recorded on the calls' streams.  bem_profile
 * clears the accumulators and switches recording on (enable != 0) or off.
 * bem_profile_read waits for the recorded events and returns the total time in
 * milliseconds and the number of launches of one kernel family (tag in
 * [0, 12): 0 sweep_f64, 1 sweep_mixed, 2 vjp_segments, 3 vjp_elements,
 * 4 features, 5 beta_rows, 6 gram_f64, 7 gram_mfma, 8 xr, 9 cholesky,
 * 10 boundary, 11 near_pairs); bem_profile_name gives the family's name (static string,
 * "" for a bad tag).  Errors: EINVAL (null context or bad tag). */
int bem_profile(bem_ctx* ctx, int32_t enable);
int bem_profile_read(bem_ctx* ctx, int32_t tag, double* total_ms, int64_t* launches);
const char* bem_profile_name(int32_t tag);

/* Release the context and every workspace it owns.  Null is ignored. */
void bem_destroy(bem_ctx* ctx);

/* Description of the last non-OK status of this context (NULL: of the last
 * failed bem_build or bem_build_elements on this thread).  Valid until the next call on the context. */
const char* bem_last_error(const bem_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* BEM_H */
