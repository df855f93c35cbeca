// Expectation operator and first-order conditions of the smooth IRBC model
// (Sec. 2.1, Table 1), the caller of the evaluation path in time iteration
// (Alg. 1): per state, the next states of every monomial-rule node are formed
// on the device, the previous policy is interpolated there by hdmr_eval's
// kernels (plain FP64), and the Euler and resource residuals are assembled
// from those values.  Conventions and formulas: include/hdmr_irbc.h.
#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/hdmr_irbc.h"
#include "kernels_common.h"

namespace hdmr {
namespace {

struct IrbcDev {
  int N, D, Q;                 // countries, shocks (N + 1), nodes 2 D
  double beta, alpha, delta, sigma, rho, phi, A;
  double gamma_lo, gamma_span;
  double a_lo, a_w, k_lo, k_w;  // box origin and width
  double r;                     // node radius sqrt(D)
};

__device__ __forceinline__ double gamma_of(const IrbcDev &P, int j) {
  return P.N > 1 ? P.gamma_lo + P.gamma_span * (double)j / (double)(P.N - 1) : P.gamma_lo;
}

// Shock values of node q on shock axis s: +r on axis q (q < D), -r on axis
// q - D (q >= D), 0 elsewhere (the degree-3 monomial rule).
__device__ __forceinline__ double node_shock(const IrbcDev &P, int q, int s) {
  const int axis = q < P.D ? q : q - P.D;
  return axis == s ? (q < P.D ? P.r : -P.r) : 0.0;
}

__device__ __forceinline__ double next_a(const IrbcDev &P, double a, int j, int q) {
  return exp(P.rho * log(a) + P.sigma * (node_shock(P, q, j) + node_shock(P, q, P.N)));
}

// Next states (row p * Q + q of Xn, 2N normalised coordinates, clipped to
// [0,1]) of states p in [p0, p0 + np).
__global__ void k_next_states(IrbcDev P, const double *__restrict__ X, const double *__restrict__ C, int64_t p0,
                              int64_t np, double *__restrict__ Xn) {
  const int d = 2 * P.N, m = P.N + 1;
  const int64_t total = np * P.Q * d;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / d;
    const int j = (int)(e - row * d);
    const int64_t p = p0 + row / P.Q;
    const int q = (int)(row % P.Q);
    double v;
    if (j < P.N) {
      const double a = P.a_lo + X[p * d + j] * P.a_w;
      v = (next_a(P, a, j, q) - P.a_lo) / P.a_w;
    } else {
      v = (C[p * m + (j - P.N)] - P.k_lo) / P.k_w;
    }
    Xn[e] = fmin(fmax(v, 0.0), 1.0);
  }
}

// Residuals of states p in [p0, p0 + np): one wavefront per state, lanes over
// countries; Pn holds the policy at the next states (row p * Q + q, m values).
__global__ __launch_bounds__(256) void k_residuals(IrbcDev P, const double *__restrict__ X,
                                                   const double *__restrict__ C, const double *__restrict__ Pn,
                                                   int64_t p0, int64_t np, double *__restrict__ R,
                                                   double *__restrict__ E) {
  const int d = 2 * P.N, m = P.N + 1;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  const double wq = 1.0 / (double)P.Q;
  for (int64_t pr = w0; pr < np; pr += nw) {
    const int64_t p = p0 + pr;
    const double lam = C[p * m + P.N];
    double res_sum = 0.0;
    for (int j = lane; j < P.N; j += WAVE) {
      const double a = P.a_lo + X[p * d + j] * P.a_w;
      const double k = P.k_lo + X[p * d + P.N + j] * P.k_w;
      const double k1 = C[p * m + j];
      const double g1 = k1 / k - 1.0;
      double ex = 0.0;
      for (int q = 0; q < P.Q; ++q) {
        const double *pn = Pn + (pr * P.Q + q) * m;
        const double a1 = next_a(P, a, j, q);
        const double g2 = pn[j] / k1 - 1.0;
        ex += wq * pn[P.N] * (a1 * P.A * P.alpha * pow(k1, P.alpha - 1.0) + (1.0 - P.delta) +
                              0.5 * P.phi * g2 * (g2 + 2.0));
      }
      R[p * m + j] = lam * (1.0 + P.phi * g1) - P.beta * ex;
      if (E) E[p * P.N + j] = ex;
      const double gam = gamma_of(P, j);
      // (lambda / tau_j)^(-gamma_j) with tau_j = A^(1/gamma_j)
      const double c = pow(lam, -gam) * P.A;
      res_sum += a * P.A * pow(k, P.alpha) + k * ((1.0 - P.delta) - 0.5 * P.phi * g1 * g1) - k1 - c;
    }
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) res_sum += __shfl_xor(res_sum, off, WAVE);
    if (lane == 0) R[p * m + P.N] = res_sum;
  }
}

}  // namespace
}  // namespace hdmr

using namespace hdmr;

extern "C" int irbc_residuals(const hdmr_model *policy, const irbc_params *params, const double *states,
                              const double *choice, int64_t n, double *residuals, double *expect,
                              hdmr_stream_t stream_) {
  clear_error();
  if (!policy || !params) return fail(HDMR_EINVAL, "irbc_residuals: null argument");
  const irbc_params &p = *params;
  if (p.N < 1 || p.N > 4096) return fail(HDMR_EINVAL, "irbc_residuals: N must be in [1, 4096]");
  if (policy->d != 2 * p.N || policy->m != p.N + 1)
    return fail(HDMR_EINVAL, "irbc_residuals: the policy model must have d = 2N and m = N + 1");
  if (!(p.a_hi > p.a_lo) || !(p.k_hi > p.k_lo) || !(p.a_lo > 0.0) || !(p.k_lo > 0.0))
    return fail(HDMR_EINVAL, "irbc_residuals: the state box must be positive and nonempty");
  if (n < 0) return fail(HDMR_EINVAL, "irbc_residuals: n must be >= 0");
  if (n == 0) return HDMR_OK;
  if (!states || !choice || !residuals) return fail(HDMR_EINVAL, "irbc_residuals: null buffer");
  int rc = set_device_of(policy);
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)stream_;
  IrbcDev P{};
  P.N = p.N;
  P.D = p.N + 1;
  P.Q = 2 * P.D;
  P.beta = p.beta;
  P.alpha = p.alpha;
  P.delta = p.delta;
  P.sigma = p.sigma;
  P.rho = p.rho;
  P.phi = p.phi;
  P.A = (1.0 - p.beta * (1.0 - p.delta)) / (p.alpha * p.beta);
  P.gamma_lo = p.gamma_lo;
  P.gamma_span = p.gamma_span;
  P.a_lo = p.a_lo;
  P.a_w = p.a_hi - p.a_lo;
  P.k_lo = p.k_lo;
  P.k_w = p.k_hi - p.k_lo;
  P.r = std::sqrt((double)P.D);
  const int d = 2 * p.N, m = p.N + 1;
  // chunks of states whose next states number at most 2^21
  const int64_t chunk = std::max<int64_t>(1, ((int64_t)1 << 21) / P.Q);
  const int64_t nc = std::min<int64_t>(n, chunk);
  double *Xn = nullptr, *Pn = nullptr;
  HDMR_HIP(dev_malloc_async((void **)&Xn, sizeof(double) * (size_t)(nc * P.Q * d), stream));
  hipError_t e = dev_malloc_async((void **)&Pn, sizeof(double) * (size_t)(nc * P.Q * m), stream);
  if (e != hipSuccess) {
    (void)hipFreeAsync(Xn, stream);
    return hip_fail(e, "irbc_residuals workspace");
  }
  for (int64_t p0 = 0; p0 < n && rc == HDMR_OK; p0 += nc) {
    const int64_t np = std::min<int64_t>(nc, n - p0);
    const int64_t tot = np * P.Q * d;
    hipLaunchKernelGGL(k_next_states, dim3((unsigned)std::min<int64_t>((tot + 255) / 256, 65536)), dim3(256), 0,
                       stream, P, states, choice, p0, np, Xn);
    if ((e = hipGetLastError()) != hipSuccess) {
      rc = hip_fail(e, "k_next_states");
      break;
    }
    rc = hdmr_eval(policy, Xn, np * P.Q, Pn, m, HDMR_PLAIN_FP64, stream);
    if (rc) break;
    hipLaunchKernelGGL(k_residuals, dim3((unsigned)std::min<int64_t>((np + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK,
                                                                    65536)),
                       dim3(256), 0, stream, P, states, choice, Pn, p0, np, residuals, expect);
    if ((e = hipGetLastError()) != hipSuccess) rc = hip_fail(e, "k_residuals");
  }
  (void)hipFreeAsync(Xn, stream);
  (void)hipFreeAsync(Pn, stream);
  return rc;
}

// ---------------------------------------------------------------------------
// Time iteration (Alg. 1) on the device: batched Newton on the first-order
// conditions with forward-difference Jacobians, a batched dense solver, and
// one time-iteration step as a build whose function is that solver.
// ---------------------------------------------------------------------------
namespace hdmr {
namespace {

constexpr int SOLVE_MAX = 64;  // largest system (N + 1) of the batched solver

// Batched dense solve J x = b (Gaussian elimination with partial pivoting),
// one wavefront per system, lane r owns row r; J (n x M x M, row-major) and b
// (n x M) are overwritten; x receives the solution (NaN rows for a singular
// system).
__global__ __launch_bounds__(64) void k_batched_solve(double *__restrict__ J, double *__restrict__ b, int64_t n,
                                                      int M, double *__restrict__ x) {
  __shared__ double s[SOLVE_MAX][SOLVE_MAX + 1];
  __shared__ double sb[SOLVE_MAX];
  const int r = threadIdx.x;
  for (int64_t sys = blockIdx.x; sys < n; sys += gridDim.x) {
    double *Js = J + sys * M * M;
    if (r < M) {
      for (int c = 0; c < M; ++c) s[r][c] = Js[(int64_t)r * M + c];
      sb[r] = b[sys * M + r];
    }
    __syncthreads();
    bool singular = false;
    for (int c = 0; c < M; ++c) {
      // pivot: the row >= c with the largest |J[row][c]| (lowest row on ties)
      double best = r >= c && r < M ? fabs(s[r][c]) : -1.0;
      int brow = r;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int orow = __shfl_xor(brow, off, 64);
        if (ob > best || (ob == best && orow < brow)) {
          best = ob;
          brow = orow;
        }
      }
      if (!(best > 0.0)) singular = true;
      if (brow != c && !singular) {
        // swap rows c and brow: lane q < M moves column q
        if (r < M) {
          const double t = s[c][r];
          s[c][r] = s[brow][r];
          s[brow][r] = t;
        }
        __syncthreads();
        if (r == 0) {
          const double t = sb[c];
          sb[c] = sb[brow];
          sb[brow] = t;
        }
      }
      __syncthreads();
      if (!singular && r > c && r < M) {
        const double f = s[r][c] / s[c][c];
        for (int q = c; q < M; ++q) s[r][q] -= f * s[c][q];
        sb[r] -= f * sb[c];
      }
      __syncthreads();
    }
    // back substitution by lane 0 (M <= 64 rows)
    if (r == 0) {
      for (int c = M - 1; c >= 0; --c) {
        double v = sb[c];
        for (int q = c + 1; q < M; ++q) v -= s[c][q] * sb[q];
        sb[c] = singular ? __builtin_nan("") : v / s[c][c];
      }
    }
    __syncthreads();
    if (r < M) x[sys * M + r] = sb[r];
    __syncthreads();
  }
}

// Stack of the Newton evaluation points: block 0 holds x, block 1 + i holds x
// with unknown i raised by its step h (per state).  Xs / Cs: (M + 1) n rows.
__global__ void k_fd_points(const double *__restrict__ X, const double *__restrict__ x, int64_t n, int d, int M,
                            double rel, double *__restrict__ Xs, double *__restrict__ Cs,
                            double *__restrict__ h) {
  const int64_t total = (int64_t)(M + 1) * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int blk = (int)(e / n);
    const int64_t p = e - (int64_t)blk * n;
    for (int j = 0; j < d; ++j) Xs[e * d + j] = X[p * d + j];
    for (int j = 0; j < M; ++j) {
      double v = x[p * M + j];
      if (blk == j + 1) {
        const double step = rel * fmax(1.0, fabs(v));
        h[p * M + j] = step;
        v += step;
      }
      Cs[e * M + j] = v;
    }
  }
}

// Jacobian columns from the stacked residuals, right-hand side -R(x), and the
// largest |R(x)| per state.
__global__ void k_fd_jacobian(const double *__restrict__ Rs, const double *__restrict__ h, int64_t n, int M,
                              double *__restrict__ J, double *__restrict__ rhs, double *__restrict__ rmax) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    double mx = 0.0;
    for (int r = 0; r < M; ++r) {
      const double r0 = Rs[p * M + r];
      rhs[p * M + r] = -r0;
      mx = fmax(mx, fabs(r0));
      if (r0 != r0) mx = __builtin_nan("");
      for (int c = 0; c < M; ++c)
        J[(p * M + r) * M + c] = (Rs[((int64_t)(c + 1) * n + p) * M + r] - r0) / h[p * M + c];
    }
    rmax[p] = mx;
  }
}

// x += dx for states whose residual is not yet below tol (others keep x).
__global__ void k_newton_update(double *__restrict__ x, const double *__restrict__ dx, const double *__restrict__ rmax,
                                int64_t n, int M, double tol) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * M; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / M;
    if (!(rmax[p] <= tol) && dx[e] == dx[e]) x[e] += dx[e];
  }
}

__global__ void k_max_reduce(const double *__restrict__ v, int64_t n, double *__restrict__ out) {
  __shared__ double part[256];
  double mx = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) mx = (v[i] != v[i] || mx != mx) ? __builtin_nan("") : fmax(mx, v[i]);
  part[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double a = part[threadIdx.x], b2 = part[threadIdx.x + s];
      part[threadIdx.x] = (a != a || b2 != b2) ? __builtin_nan("") : fmax(a, b2);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

// Euler-equation errors of a policy: unit-free |R_j| / (lambda (1 + phi g_j))
// for the N Euler conditions and |R_N| / sum_j c_j for the resource
// constraint, with the choice taken from the policy itself at the states.
__global__ void k_euler_errors(IrbcDev P, const double *__restrict__ X, const double *__restrict__ C,
                               const double *__restrict__ R, int64_t n, double *__restrict__ err) {
  const int d = 2 * P.N, m = P.N + 1;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const double lam = C[p * m + P.N];
    double csum = 0.0;
    for (int j = 0; j < P.N; ++j) {
      const double k = P.k_lo + X[p * d + P.N + j] * P.k_w;
      const double g1 = C[p * m + j] / k - 1.0;
      err[p * m + j] = fabs(R[p * m + j]) / fabs(lam * (1.0 + P.phi * g1));
      csum += pow(lam, -gamma_of(P, j)) * P.A;
    }
    err[p * m + P.N] = fabs(R[p * m + P.N]) / csum;
  }
}

IrbcDev make_dev(const irbc_params &p) {
  IrbcDev P{};
  P.N = p.N;
  P.D = p.N + 1;
  P.Q = 2 * P.D;
  P.beta = p.beta;
  P.alpha = p.alpha;
  P.delta = p.delta;
  P.sigma = p.sigma;
  P.rho = p.rho;
  P.phi = p.phi;
  P.A = (1.0 - p.beta * (1.0 - p.delta)) / (p.alpha * p.beta);
  P.gamma_lo = p.gamma_lo;
  P.gamma_span = p.gamma_span;
  P.a_lo = p.a_lo;
  P.a_w = p.a_hi - p.a_lo;
  P.k_lo = p.k_lo;
  P.k_w = p.k_hi - p.k_lo;
  P.r = std::sqrt((double)P.D);
  return P;
}

unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

}  // namespace
}  // namespace hdmr

extern "C" int irbc_solve(const hdmr_model *policy, const irbc_params *params, const double *states, double *x,
                          int64_t n, int32_t max_iter, double tol, int32_t *iters, double *max_residual,
                          hdmr_stream_t stream_) {
  clear_error();
  if (!policy || !params || (n > 0 && (!states || !x))) return fail(HDMR_EINVAL, "irbc_solve: null argument");
  if (max_iter < 0 || !(tol >= 0.0)) return fail(HDMR_EINVAL, "irbc_solve: max_iter >= 0 and tol >= 0 required");
  const int N = params->N, M = N + 1, d = 2 * N;
  if (N < 1 || M > SOLVE_MAX) return fail(HDMR_EUNSUPPORTED, "irbc_solve: N must be in [1, 63]");
  if (iters) *iters = 0;
  if (max_residual) *max_residual = 0.0;
  if (n == 0) return HDMR_OK;
  int rc = set_device_of(policy);
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)stream_;
  const int64_t ns = (int64_t)(M + 1) * n;
  double *Xs = nullptr, *Cs = nullptr, *Rs = nullptr, *h = nullptr, *J = nullptr, *rhs = nullptr, *dx = nullptr,
         *rmax = nullptr, *dmax = nullptr;
  size_t bytes[] = {sizeof(double) * (size_t)(ns * d), sizeof(double) * (size_t)(ns * M),
                    sizeof(double) * (size_t)(ns * M), sizeof(double) * (size_t)(n * M),
                    sizeof(double) * (size_t)(n * M * M), sizeof(double) * (size_t)(n * M),
                    sizeof(double) * (size_t)(n * M), sizeof(double) * (size_t)n, sizeof(double)};
  double **ptrs[] = {&Xs, &Cs, &Rs, &h, &J, &rhs, &dx, &rmax, &dmax};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 9 && e == hipSuccess; ++i) e = dev_malloc_async((void **)ptrs[i], bytes[i], stream);
  auto release = [&]() {
    for (double **p : ptrs)
      if (*p) (void)hipFreeAsync(*p, stream);
  };
  if (e != hipSuccess) {
    release();
    return hip_fail(e, "irbc_solve workspace");
  }
  const double rel = 1e-7;  // forward-difference step relative to max(1, |x|)
  double worst = 0.0;
  int it = 0;
  for (;; ++it) {
    hipLaunchKernelGGL(k_fd_points, dim3(grid1(ns)), dim3(256), 0, stream, states, x, n, d, M, rel, Xs, Cs, h);
    if ((rc = irbc_residuals(policy, params, Xs, Cs, ns, Rs, nullptr, stream))) break;
    hipLaunchKernelGGL(k_fd_jacobian, dim3(grid1(n)), dim3(256), 0, stream, Rs, h, n, M, J, rhs, rmax);
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, stream, rmax, n, dmax);
    if ((e = hipMemcpyAsync(&worst, dmax, sizeof(double), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess) {
      rc = hip_fail(e, "irbc_solve");
      break;
    }
    if (worst <= tol || it >= max_iter) break;
    hipLaunchKernelGGL(k_batched_solve, dim3((unsigned)std::min<int64_t>(n, 65536)), dim3(64), 0, stream, J, rhs, n,
                       M, dx);
    hipLaunchKernelGGL(k_newton_update, dim3(grid1(n * M)), dim3(256), 0, stream, x, dx, rmax, n, M, tol);
    if ((e = hipGetLastError()) != hipSuccess) {
      rc = hip_fail(e, "irbc_solve");
      break;
    }
  }
  release();
  if (iters) *iters = it;
  if (max_residual) *max_residual = worst;
  return rc;
}

extern "C" int irbc_euler_errors(const hdmr_model *policy, const irbc_params *params, const double *states, int64_t n,
                                 double *errors, hdmr_stream_t stream_) {
  clear_error();
  if (!policy || !params || (n > 0 && (!states || !errors))) return fail(HDMR_EINVAL, "irbc_euler_errors: null argument");
  const int N = params->N, M = N + 1;
  if (n == 0) return HDMR_OK;
  if (policy->d != 2 * N || policy->m != M)
    return fail(HDMR_EINVAL, "irbc_euler_errors: the policy model must have d = 2N and m = N + 1");
  int rc = set_device_of(policy);
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)stream_;
  double *C = nullptr, *R = nullptr;
  HDMR_HIP(dev_malloc_async((void **)&C, sizeof(double) * (size_t)(n * M), stream));
  hipError_t e = dev_malloc_async((void **)&R, sizeof(double) * (size_t)(n * M), stream);
  if (e != hipSuccess) {
    (void)hipFreeAsync(C, stream);
    return hip_fail(e, "irbc_euler_errors workspace");
  }
  rc = hdmr_eval(policy, states, n, C, M, HDMR_PLAIN_FP64, stream);
  if (!rc) rc = irbc_residuals(policy, params, states, C, n, R, nullptr, stream);
  if (!rc) {
    hipLaunchKernelGGL(k_euler_errors, dim3(grid1(n)), dim3(256), 0, stream, make_dev(*params), states, C, R, n,
                       errors);
    if ((e = hipGetLastError()) != hipSuccess) rc = hip_fail(e, "k_euler_errors");
  }
  (void)hipFreeAsync(C, stream);
  (void)hipFreeAsync(R, stream);
  return rc;
}

namespace {
struct StepCtx {
  const hdmr_model *prev;
  const irbc_params *params;
  int32_t max_iter;
  double tol;
  int32_t worst_iters;
  double worst_residual;
  int rc;
};

// The build's function: the FOC solution at every requested state, started
// from the previous policy there.
int solve_callback(const double *X, int64_t n, int32_t d, double *Y, int32_t m, void *user) {
  StepCtx &S = *static_cast<StepCtx *>(user);
  double *dX = nullptr, *dY = nullptr;
  hipStream_t st = (hipStream_t)0;
  if (dev_malloc((void **)&dX, sizeof(double) * (size_t)(n * d)) != hipSuccess) return -1;
  if (dev_malloc((void **)&dY, sizeof(double) * (size_t)(n * m)) != hipSuccess) {
    (void)hipFree(dX);
    return -1;
  }
  int rc = hipMemcpy(dX, X, sizeof(double) * (size_t)(n * d), hipMemcpyHostToDevice) == hipSuccess ? 0 : HDMR_EDEVICE;
  if (!rc) rc = hdmr_eval(S.prev, dX, n, dY, m, HDMR_PLAIN_FP64, st);
  int32_t it = 0;
  double worst = 0.0;
  if (!rc) rc = irbc_solve(S.prev, S.params, dX, dY, n, S.max_iter, S.tol, &it, &worst, st);
  if (!rc && hipMemcpy(Y, dY, sizeof(double) * (size_t)(n * m), hipMemcpyDeviceToHost) != hipSuccess) rc = HDMR_EDEVICE;
  (void)hipFree(dX);
  (void)hipFree(dY);
  S.worst_iters = std::max(S.worst_iters, it);
  S.worst_residual = std::max(S.worst_residual, worst);
  if (rc) S.rc = rc;
  return rc ? -1 : 0;
}
}  // namespace

extern "C" int irbc_time_step(const hdmr_model *prev, const irbc_params *params, const asg_build_params *build,
                              int32_t max_iter, double tol, hdmr_model **out, int32_t *iters, double *max_residual) {
  clear_error();
  if (!prev || !params || !build || !out) return fail(HDMR_EINVAL, "irbc_time_step: null argument");
  *out = nullptr;
  const int N = params->N;
  if (prev->d != 2 * N || prev->m != N + 1 || build->d != 2 * N || build->m != N + 1)
    return fail(HDMR_EINVAL, "irbc_time_step: models must have d = 2N and m = N + 1");
  StepCtx S{prev, params, max_iter, tol, 0, 0.0, HDMR_OK};
  int rc = asg_build_components(build, solve_callback, &S, out);
  if (iters) *iters = S.worst_iters;
  if (max_residual) *max_residual = S.worst_residual;
  if (rc == HDMR_ECALLBACK && S.rc) {
    const std::string inner = hdmr_last_error();
    return fail(S.rc, "irbc_time_step: FOC solve failed: " + inner);
  }
  return rc;
}
