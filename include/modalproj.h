/*
 * modalproj.h -- C ABI of the MI355X separable bispectrum projection.
 *
 * The library computes the matrix Gamma' of the separable ("2D") form of
 * the modal projection: Sec. 2.2, Eq. (2D) with P_ii'(r, mu) from
 * Eq. (legendre), and the projected primordial modes of the Appendix
 * (qt_i(r, l) = Int dk k^2 qbar_i(k) Delta_l(k) j_l(k r)).  Names used in
 * this header:
 *
 *   q_p(k)      primordial 1-D mode p  (the Appendix's qbar_i(k)), p < np
 *   qbar_a(l)   late-time 1-D mode a   (the Appendix's q_i(l)),    a < na
 *   beta_p(l,r) = (2/pi) Sum_k wk k^2 q_p(k) Delta_l(k) j_l(k r)
 *               (the Appendix's qt_p(r, l), times 2/pi)
 *   w_l         = (2l+1)^(1 - v_power) / sqrt(C_l); v_power = 1/6 gives
 *               the (2l+1)/(v_l sqrt(C_l)) of Eq. (legendre) with
 *               v_l = (2l+1)^(1/6) (Appendix)
 *   S_ap(r,mu)  = Sum_l w_l qbar_a(l) beta_p(l, r) P_l(mu)
 *               (Eq. (legendre)'s P_ii'(r, mu), a <-> i, p <-> i')
 *   W(r,mu)     = wr_r r^2 wmu_mu   (the r^2 dr and dmu measures)
 *
 * and Gamma is returned in one of two forms:
 *
 *   ORDERED   Gamma[A][P] = 1/(8 pi) Sum_r Sum_mu W S_{a1p1} S_{a2p2} S_{a3p3}
 *             for A = tri_a[row] = (a1,a2,a3), P = tri_p[col] = (p1,p2,p3)
 *   SYMMETRIC Gamma[n][m] = 1/(48 pi) Sum_r Sum_mu W perm[S_{a_s p_t}]
 *             (Eq. (2D): the six permutation products of the 3x3 block,
 *             i.e. its permanent; repeated indices keep all six terms)
 *
 * Beside Gamma' it computes the late-time Gram matrix <Q_n, Q_m> and the
 * full Gamma = <Q, Q>^-1 Gamma' of the Appendix (modal_gram,
 * modal_gamma_modal), Gamma' by the direct sum over l-triples of Eq. (3D)
 * with no mu integral (modal_gamma_3d), the adjoint of Gamma'
 * (modal_gamma_backward) and host-side weights of the r rules
 * (modal_r_weights).
 *
 * The mu sum of every r is completed before it enters the r sum (Sec. 2.2).
 * l runs over lmin..lmax (Eq. (3D) starts at l = 2); the arrays indexed
 * by l hold L = lmax - lmin + 1 rows.
 *
 * Memory.  Every array argument may be host memory or device memory of the
 * context's device; the library detects which.  All floating-point arrays
 * are FP64, all index arrays int32, every layout row-major (C order).  The
 * caller owns all inputs and outputs; the library keeps no pointer after a
 * call returns.  Device-memory outputs are complete once the context's
 * stream reaches the end of the call's work; host-memory outputs are
 * complete when the call returns (the library synchronises the stream).
 * The context owns a device workspace that grows on demand and is released
 * by modal_destroy.
 *
 * Errors.  Nothing is thrown and nothing aborts across this boundary: each
 * call returns a modal_status, and modal_last_error() gives a message for
 * the last failing call on that context.  A context is not thread-safe;
 * separate contexts are independent.
 */
#ifndef MODALPROJ_H
#define MODALPROJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct modal_ctx_s *modal_ctx;

typedef enum {
    MODAL_OK = 0,
    MODAL_ERR_INVALID_ARG = 1,   /* NULL pointer, bad enum, bad option        */
    MODAL_ERR_SHAPE = 2,         /* sizes/indices out of range                 */
    MODAL_ERR_OOM = 3,           /* device allocation failed or over the cap   */
    MODAL_ERR_DEVICE = 4,        /* no usable device, or a HIP runtime error   */
    MODAL_ERR_NUMERIC = 5,       /* non-positive C_l, non-finite input         */
    MODAL_ERR_UNSUPPORTED = 6    /* valid request the library does not handle  */
} modal_status;

/* Arithmetic of the projection.
 *   MODAL_FP64  : every stage in FP64 (j_l, P_l, beta, S, Gamma).
 *   MODAL_MIXED : j_l, P_l, beta and S in FP64; the triple-product quadrature
 *                 of Eq. (2D) on BF16 matrix cores with each operand split in
 *                 a high and a low BF16 part (three products per term),
 *                 FP32 accumulation of each r's mu sum and FP64 accumulation
 *                 of the r sum. */
typedef enum { MODAL_FP64 = 0, MODAL_MIXED = 1 } modal_precision;

typedef enum { MODAL_GAMMA_ORDERED = 0, MODAL_GAMMA_SYMMETRIC = 1 } modal_gamma_kind;

/* Rules for the integral over r (modal_r_weights). */
typedef enum { MODAL_R_TRAPEZOID = 0, MODAL_R_HERMITE = 1 } modal_r_rule;

/* The Wigner symbol in h^2 for Eq. (3D) (modal_gamma_3d). */
typedef enum { MODAL_3J_EXACT = 0, MODAL_3J_GOSPER = 1 } modal_threej;

/* Quadrature grids.  k ascending > 0; r > 0.  wk and wr are the weights of
 * the k and r rules (the r^2 of Eq. (2D) is applied by the library).  If
 * mu and wmu are both NULL the library computes the nmu-point
 * Gauss-Legendre rule itself.  Unless allow_inexact_gl is non-zero, nmu
 * must be at least ceil((3 lmax + 1) / 2), the smallest rule that
 * integrates P_l1 P_l2 P_l3 exactly (Sec. 2.2). */
typedef struct {
    int32_t lmin, lmax;
    int32_t nk;
    const double *k, *wk;      /* [nk] */
    int32_t nr;
    const double *r, *wr;      /* [nr] */
    int32_t nmu;
    const double *mu, *wmu;    /* [nmu] or both NULL */
    int32_t allow_inexact_gl;
} modal_grid;

/* Transfer table, power spectrum, the two 1-D bases and the mode lists. */
typedef struct {
    const double *delta;       /* Delta_l(k)   [L][nk]                      */
    const double *cl;          /* C_l          [L], every entry > 0         */
    int32_t np;
    const double *qk;          /* q_p(k)       [np][nk]                     */
    int32_t na;
    const double *ql;          /* qbar_a(l)    [na][L]                      */
    double v_power;            /* exponent of v_l; 1/6 in the paper         */
    int32_t kind;              /* modal_gamma_kind                          */
    int32_t ta;
    const int32_t *tri_a;      /* [ta][3] late-time triples, entries < na   */
    int32_t tp;
    const int32_t *tri_p;      /* [tp][3] primordial triples, entries < np  */
} modal_problem;

/* ------------------------------------------------------------------ */
/* Context                                                            */
/* ------------------------------------------------------------------ */

/* Create a context on HIP device `device`, enqueueing its work on
 * `hip_stream` (a hipStream_t; NULL = the device's null stream).
 * Returns MODAL_ERR_DEVICE if the device cannot be used. */
modal_status modal_create(modal_ctx *out, int device, void *hip_stream);

/* Release the context and its workspace (waits for its stream). */
modal_status modal_destroy(modal_ctx ctx);

/* Change the stream later calls enqueue on. */
modal_status modal_set_stream(modal_ctx ctx, void *hip_stream);

/* Static text for a status code. */
const char *modal_status_str(modal_status s);

/* Message of the last failing call on ctx (on any context if ctx is NULL);
 * valid until the next call on that context. */
const char *modal_last_error(modal_ctx ctx);

/* Cap on the workspace in bytes (0 = no cap).  A call that would need more
 * returns MODAL_ERR_OOM. */
modal_status modal_set_workspace_limit(modal_ctx ctx, size_t bytes);

/* Reuse of the forward tables by modal_gamma_backward (off by default).
 * When on, modal_gamma_backward takes the tables of steps a-c (the GL rule,
 * P_l, the weights and the scaled S rows) from the context instead of
 * recomputing them, if the context's previous call was modal_gamma or
 * modal_gamma_backward with the same grid and problem: every field equal,
 * pointers included.  The caller guarantees that the arrays behind those
 * pointers have not changed since that call; any other call in between
 * (except modal_set_forward_reuse, modal_set_workspace_limit,
 * modal_enable_timing, modal_stage_times and modal_workspace_bytes) makes the
 * backward recompute them.  The adjoint of the k contraction regenerates
 * j_l either way. */
modal_status modal_set_forward_reuse(modal_ctx ctx, int on);

/* Device bytes the context would hold for modal_gamma on this problem. */
modal_status modal_workspace_bytes(modal_ctx ctx, const modal_grid *grid,
                                   const modal_problem *prob, modal_precision prec,
                                   size_t *bytes);

/* Stage timing.  When enabled, each later call records HIP events around
 * its kernels on the context's stream; modal_stage_times then waits for the
 * stream and reports the milliseconds of the last call's stages, in order
 * MODAL_STAGE_GL, _LEGENDRE, _BESSEL, _BETA, _S, _TRIPLE, _GATHER, the
 * adjoint's _ADJ_TRIPLE, _ADJ_S, _ADJ_BETA, then _PREP (operand conversion
 * before the mixed triple product) and _ADJ_PREP (the adjoint's operand
 * assembly before _ADJ_TRIPLE); 0 for a stage the call did not run.  The
 * _TRIPLE and _ADJ_TRIPLE times cover the triple-product kernels alone.
 * n is the length of ms (>= MODAL_NSTAGES). */
enum { MODAL_STAGE_GL = 0, MODAL_STAGE_LEGENDRE, MODAL_STAGE_BESSEL, MODAL_STAGE_BETA,
       MODAL_STAGE_S, MODAL_STAGE_TRIPLE, MODAL_STAGE_GATHER,
       MODAL_STAGE_ADJ_TRIPLE, MODAL_STAGE_ADJ_S, MODAL_STAGE_ADJ_BETA,
       MODAL_STAGE_PREP, MODAL_STAGE_ADJ_PREP, MODAL_NSTAGES };
modal_status modal_enable_timing(modal_ctx ctx, int on);
modal_status modal_stage_times(modal_ctx ctx, double *ms, int n);
/* How many timed intervals each stage of the last call recorded (stages
 * that run in chunks record one per chunk: the Bessel/beta l chunks, and the
 * r batches of modal_gamma_3d under _PREP); 0 when timing is off.  Does not
 * wait for the stream.  n is the length of counts (>= MODAL_NSTAGES). */
modal_status modal_stage_counts(modal_ctx ctx, int32_t *counts, int n);

/* ------------------------------------------------------------------ */
/* Stage entry points (step a)                                        */
/* ------------------------------------------------------------------ */

/* n-point Gauss-Legendre rule on [-1, 1] (Sec. 2.2: exact for the
 * polynomial mu integrand).  x ascending, x[i] = -x[n-1-i]; w > 0.
 * x, w: [n].  n >= 1.  Each root is refined by Newton's method in
 * double-double arithmetic and rounded once (nodes and weights correctly
 * rounded to FP64).  With ctx == NULL the rule is computed on the host, into
 * host arrays, by the same code (no context and no device needed; errors
 * are read with modal_last_error(NULL)); otherwise on the context's device
 * (host or device arrays, as everywhere). */
modal_status modal_gauss_legendre(modal_ctx ctx, int32_t n, double *x, double *w);

/* Legendre table P[l][j] = P_l(mu_j), l = 0..lmax, j < nmu (the P_l(mu) of
 * Eq. (legendre)).  mu: [nmu] in [-1, 1]; P: [lmax+1][nmu]. */
modal_status modal_legendre_table(modal_ctx ctx, int32_t lmax, int32_t nmu,
                                  const double *mu, double *P);

/* Spherical Bessel table J[l][i] = j_l(x_i), l = 0..lmax (the j_l(kr) of
 * the projected modes, Appendix).  x: [nx], every x_i >= 0;
 * J: [lmax+1][nx]. */
modal_status modal_sph_bessel_table(modal_ctx ctx, int32_t lmax, int64_t nx,
                                    const double *x, double *J);

/* ------------------------------------------------------------------ */
/* Stage entry points (steps b, c, d)                                 */
/* ------------------------------------------------------------------ */

/* beta_p(l, r) (Appendix, projected modes, times 2/pi).
 * beta: [np][L][nr].  Uses grid k, wk, r and prob delta, qk. */
modal_status modal_beta(modal_ctx ctx, const modal_grid *grid, const modal_problem *prob,
                        modal_precision prec, double *beta);

/* S_ap(r, mu) of Eq. (legendre) from a given beta ([np][L][nr]).
 * S: [na][np][nr][nmu]. */
modal_status modal_S(modal_ctx ctx, const modal_grid *grid, const modal_problem *prob,
                     modal_precision prec, const double *beta, double *S);

/* Gamma of Eq. (2D) (ordered or symmetric, per prob->kind) from a given S
 * ([na][np][nr][nmu]).  gamma: [ta][tp]. */
modal_status modal_gamma_from_S(modal_ctx ctx, const modal_grid *grid,
                                const modal_problem *prob, modal_precision prec,
                                const double *S, double *gamma);

/* The whole projection: grids -> P_l, j_l -> beta -> S -> Gamma.
 * gamma: [ta][tp]. */
modal_status modal_gamma(modal_ctx ctx, const modal_grid *grid, const modal_problem *prob,
                         modal_precision prec, double *gamma);

/* The late-time Gram matrix <Q_n, Q_m> of the inner product of Sec. 2.1
 * (weights h^2 / (v1 v2 v3)^2), between the late-time modes of tri_a and
 * themselves: gram [ta][ta], symmetric.  With h^2 as the Gauss-Legendre mu
 * integral (Sec. 2.2) it takes the form of Eq. (2D) with
 * G_ab(mu) = Sum_l (2l+1) / v_l^2 qbar_a(l) qbar_b(l) P_l(mu) in place of
 * P_ii'(r, mu) and no r integral; the same kernels compute it.  Reads the l
 * range, nmu (and mu, wmu if given) of the grid, and na, ql, v_power, kind,
 * ta and tri_a of the problem (cl, np, qk, delta and tri_p are not used, but
 * cl must be valid).  na * na <= 8192.  Precision as for modal_gamma. */
modal_status modal_gram(modal_ctx ctx, const modal_grid *grid, const modal_problem *prob,
                        modal_precision prec, double *gram);

/* The full projection matrix Gamma = <Q, Q>^-1 <Q, Q~> (Appendix):
 * gamma [ta][tp] = gram^-1 Gamma', with Gamma' as modal_gamma computes it in
 * the given precision and gram = <Q, Q> over tri_a (modal_gram) in FP64,
 * solved by a Cholesky factorisation (rocSOLVER) and two triangular solves
 * (rocBLAS).  MODAL_ERR_NUMERIC if the Gram matrix is not positive definite
 * in FP64: late-time modes that are linearly dependent, or so nearly so that
 * rounding makes a pivot non-positive (products of polynomials in l of total
 * degree above about 25, restricted to the triangle condition, reach that at
 * lmax in the thousands).  The result's rounding grows with the condition
 * number of <Q, Q>.  The workspace holds gram besides the forward's. */
modal_status modal_gamma_modal(modal_ctx ctx, const modal_grid *grid, const modal_problem *prob,
                               modal_precision prec, double *gamma);

/* The size in bytes of the device scratch array behind modal_gamma_noalloc
 * (one per device, held until the process ends). */
#define MODAL_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): Gamma
 * exactly as modal_gamma computes it (same kernels, same results), with
 * every intermediate buffer and plan taken from a fixed device scratch array
 * of MODAL_NOALLOC_SCRATCH_BYTES per device instead of the context's
 * workspace; the call makes no hipMalloc or hipFree (nor any allocating
 * library call).  Every array, gamma included, must be device memory of the
 * context's device (MODAL_ERR_INVALID_ARG otherwise: a host array would need
 * staging).  A problem whose buffers do not fit in the scratch is refused
 * with MODAL_ERR_OOM before its triple product runs (modal_gamma takes any
 * size); the lmax = 64, 512 x 512 workload fits in either precision.  Stage
 * timing is not recorded, and the adjoint cannot reuse this call's tables.
 * All calls on one device share its scratch, which keeps the last call's
 * contents: calls that overlap on one device (other contexts, other streams)
 * race.  Validation still reads C_l and the mode lists back to the host. */
modal_status modal_gamma_noalloc(modal_ctx ctx, const modal_grid *grid, const modal_problem *prob,
                                 modal_precision prec, double *gamma);

/* Gamma' of Eq. (3D) (Modal3D): the direct sum over l-triples with the
 * weight h^2 of Sec. 2.1 (Eq. (weight-function)) taken from the Wigner symbol
 * itself, MODAL_3J_EXACT (exact, by a product recurrence in FP64), or from
 * the Gosper approximation that Eq. (3D) prints (MODAL_3J_GOSPER, within
 * 2.3 % of the exact symbol for l >= 2), and no mu integral: the form the
 * paper keeps for bases where the separable form is unstable.  With the exact
 * symbol it equals modal_gamma's Gamma' up to rounding.  Same grid and
 * problem as modal_gamma (mu, wmu unused, nmu only validated as >= 1; both
 * kinds); FP64 throughout; host or device arrays as everywhere.
 * np * na = U <= 1280.  Workspace: the moment tensor over u1 and the pairs
 * u2 <= u3, 4 U^2 (U + 1) bytes, beta and the Bessel chunks as in the
 * forward, and the operands of one batch of nb radial points,
 * 8 nb (2 L U + U (U + 1) / 2 + U) bytes.  r is taken in balanced
 * batches of at most the count whose operands fit in 8 GiB, or in a quarter
 * of the workspace limit when one is set.  gamma: [ta][tp]. */
modal_status modal_gamma_3d(modal_ctx ctx, const modal_grid *grid, const modal_problem *prob,
                            int32_t threej, double *gamma);

/* Weights w[j] of a rule for the integral of y(r) over [r[0], r[n-1]] on
 * the given nodes, sum_j w[j] y[j]; they go into modal_grid.wr (the library
 * multiplies by r^2 itself).  Host arrays, no context, no device work.
 *   MODAL_R_TRAPEZOID: the trapezium rule (the rule the paper's timings use,
 *     Modal3D algorithmic change).
 *   MODAL_R_HERMITE: the local Hermite-cubic integrator of Eq. (hermite):
 *     on each interval the cubic Hermite interpolant of y, with the
 *     derivative at r_k taken as the slope of the chord from r_k to r_{k+1},
 *     integrated exactly.  Eq. (hermite) is read with the factor
 *     (r_{k+1} - r_k) on both derivative terms (it is printed on the first
 *     only); at the last node the derivative is the slope of the last chord,
 *     so the last interval reduces to the trapezium.  Exact for linear y.
 * n >= 2 and r strictly ascending, else MODAL_ERR_SHAPE; non-finite r is
 * MODAL_ERR_NUMERIC; an unknown rule or a NULL pointer MODAL_ERR_INVALID_ARG.
 * The message is read with modal_last_error(NULL). */
modal_status modal_r_weights(int32_t rule, int32_t n, const double *r, double *w);

/* Gradient of a scalar loss L of Gamma (the adjoint of modal_gamma, with the
 * same grid and problem): given dgamma = dL/dGamma ([ta][tp]), writes
 * dqk = dL/dq_p(k) ([np][nk]) and ddelta = dL/dDelta_l(k) ([L][nk]); either
 * output may be NULL.  Every stage of the forward (Eq. (2D), Eq. (legendre),
 * the Appendix's projected modes) is differentiated in reverse order; the
 * j_l tables are regenerated, never stored.  The mode lists must not repeat a
 * triple (for SYMMETRIC: a sorted triple), else MODAL_ERR_SHAPE.
 * MODAL_FP64 runs every adjoint stage in FP64; MODAL_MIXED runs the adjoint
 * of Eq. (2D) (dL/dS from dL/dGamma, the dominant stage) on BF16 matrix cores
 * with split operands, FP32 partial sums (over the w of one v, then over 64
 * values of v) and FP64 accumulation, and the other adjoint stages in FP64.
 * The workspace holds, besides the forward's, dL/dS (as large as S) and the
 * tensor dL/dT in blocks (about 4 U^3 bytes for FP64, 2 U^3 for MIXED,
 * U = np * na). */
modal_status modal_gamma_backward(modal_ctx ctx, const modal_grid *grid,
                                  const modal_problem *prob, modal_precision prec,
                                  const double *dgamma, double *dqk, double *ddelta);

#ifdef __cplusplus
}
#endif

#endif /* MODALPROJ_H */
