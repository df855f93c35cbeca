/*
 * hdmr_irbc.h -- the expectation operator of time iteration and the
 * first-order conditions of the smooth international real business cycle
 * (IRBC) model (Sec. 2.1, Table 1; time iteration Alg. 1, Sec. 2.2), with the
 * previous policy held as an HDMR sparse-grid model (hdmr.h) and every
 * expectation taken over next states evaluated by hdmr_eval's kernels.
 *
 * Model (N countries, state x_t = (a_t, k_t) in R^{2N}, policy
 * p(x_t) = (k_{t+1}, lambda_t) in R^{N+1}):
 *   ln a_{j,t+1} = rho ln a_{j,t} + sigma (e_{j,t+1} + e_{t+1}), e ~ N(0, 1)
 *   (N country shocks and one global shock, independent);
 *   Euler condition of country j (eq (model1)):
 *     lambda_t (1 + phi g_{j,t+1}) - beta E_t[ lambda_{t+1} ( a_{j,t+1} A alpha
 *       k_{j,t+1}^(alpha-1) + 1 - delta + phi/2 g_{j,t+2} (g_{j,t+2} + 2) ) ] = 0,
 *     g_{j,t+1} = k_{j,t+1} / k_{j,t} - 1;
 *   aggregate resource constraint (eq (model2)):
 *     sum_j ( a_{j,t} A k_{j,t}^alpha + k_{j,t} ((1 - delta) - phi/2 g_{j,t+1}^2)
 *             - k_{j,t+1} - (lambda_t / tau_j)^(-gamma_j) ) = 0,
 *   A = (1 - beta (1 - delta)) / (alpha beta), tau_j = A^(1/gamma_j),
 *   gamma_j = gamma_lo + gamma_span (j - 1) / (N - 1)  (gamma_lo for N = 1).
 * E_t is the degree-3 monomial rule over the N + 1 shocks (2 (N + 1) nodes
 * +-sqrt(N + 1) along each shock axis, weights 1 / (2 (N + 1))).
 *
 * The policy model maps normalised states in [0,1]^{2N} (x = (a - a_lo) /
 * (a_hi - a_lo) for the first N coordinates, (k - k_lo) / (k_hi - k_lo) for
 * the last N) to (k_{t+1}, lambda_t) in model units (m = N + 1).  Next states
 * are clipped to the box before they are interpolated; the integrand uses
 * the unclipped a_{j,t+1}.
 *
 * Conventions as in hdmr.h (return codes, hdmr_last_error, asynchronous
 * calls on the given stream, caller-owned buffers).
 */
#ifndef HDMR_IRBC_H
#define HDMR_IRBC_H

#include "hdmr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t N;                          /* countries: d = 2N state, m = N + 1 policy   */
  double beta, alpha, delta, sigma, rho, phi;  /* Table 1                            */
  double gamma_lo, gamma_span;        /* gamma_j = gamma_lo + gamma_span (j-1)/(N-1) */
  double a_lo, a_hi, k_lo, k_hi;      /* state box mapped to [0,1]^{2N}              */
} irbc_params;

/* FOC residuals at n states for candidate policy values.
 *   policy    : previous policy p~ (d = 2N, m = N + 1), evaluated at the
 *               2 (N + 1) n next states in plain FP64;
 *   states    : dev, n x 2N normalised states x_t;
 *   choice    : dev, n x (N + 1): k_{t+1} (N values, model units), lambda_t;
 *   residuals : dev, n x (N + 1): the N Euler residuals, then the resource
 *               constraint;
 *   expect    : dev, n x N or NULL: the expectations E_t[...] of the Euler
 *               conditions.
 * The next states and their policy values live in a workspace the call
 * allocates (stream-ordered) and frees; large n is processed in chunks.
 * HDMR_EINVAL on shape mismatch (policy d != 2N or m != N + 1), N < 1,
 * a non-positive or empty box, or k_{t+1} <= 0 rows are not checked (they
 * give NaN residuals). */
int irbc_residuals(const hdmr_model *policy, const irbc_params *params, const double *states, const double *choice,
                   int64_t n, double *residuals, double *expect, hdmr_stream_t stream);

/* Batched Newton solve of the first-order conditions (the FOC solve of
 * Alg. 1, step 4, in place of IPOPT): for each of n states, find
 * x = (k_{t+1}, lambda_t) with irbc_residuals(policy, ..., x) = 0.
 *   x (dev, n x (N + 1)): in, the starting guess; out, the iterate at exit.
 * Each iteration evaluates the residuals at x and at N + 1 forward-difference
 * points (unknown i raised by 1e-7 max(1, |x_i|)) in one stacked call, solves
 * the (N + 1) x (N + 1) systems J dx = -R by Gaussian elimination with partial
 * pivoting (one wavefront per system), and updates the states whose largest
 * |residual| exceeds tol.  Stops when every state's largest |residual| is
 * <= tol or after max_iter updates; *iters (may be NULL) receives the updates
 * made and *max_residual (may be NULL) the largest |residual| at x on exit.
 * Synchronises the stream once per iteration.  N <= 63 (HDMR_EUNSUPPORTED
 * beyond). */
int irbc_solve(const hdmr_model *policy, const irbc_params *params, const double *states, double *x, int64_t n,
               int32_t max_iter, double tol, int32_t *iters, double *max_residual, hdmr_stream_t stream);

/* Unit-free Euler-equation errors of a policy at n states (Sec. 5): the
 * choice is the policy's own value at each state and the next-period policy
 * is the same model; errors (dev, n x (N + 1)) receive |R_j| / |lambda_t
 * (1 + phi g_{j,t+1})| for the N Euler conditions and |R_N| / sum_j c_j for
 * the resource constraint (c_j = (lambda_t / tau_j)^(-gamma_j)). */
int irbc_euler_errors(const hdmr_model *policy, const irbc_params *params, const double *states, int64_t n,
                      double *errors, hdmr_stream_t stream);

/* One time-iteration step (Alg. 1, steps 2-5): a new policy model built with
 * asg_build_components(build, f) where f, at the build's nodes, is the FOC
 * solution (irbc_solve with max_iter, tol) started from the previous policy
 * prev at those states.  build->d must be 2N and build->m N + 1.  *iters and
 * *max_residual (may be NULL) receive the largest Newton iteration count and
 * final residual over the build's solves.  Synchronous. */
int irbc_time_step(const hdmr_model *prev, const irbc_params *params, const asg_build_params *build,
                   int32_t max_iter, double tol, hdmr_model **out, int32_t *iters, double *max_residual);

#ifdef __cplusplus
}
#endif

#endif /* HDMR_IRBC_H */
