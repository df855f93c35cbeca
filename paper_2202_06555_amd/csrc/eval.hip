// Evaluation of F(x) = c0 + sum_S w_S u_S(x_S) and of its gradient, FP64.
//
// One wavefront owns one point at a time:
//   stage   : the point's d coordinates go to LDS (read once from HBM);
//   lookup  : lanes run over the model's level multi-indices ("tuples"), 64
//             at a time; for its tuple a lane computes the active cell of
//             every dimension (the single odd index whose support holds x,
//             eq (3.3)), the basis product w = w_S prod phi (eq (3.1),
//             eq (3.2)) and the row of that cell through the directory;
//   compact : a wave ballot + prefix count packs the hits (row, w) into a
//             64-entry LDS queue;
//   contract: lanes run over outputs (several hits per instruction when m
//             is small) and accumulate w * alpha[row, o] in FP64 registers,
//             coalesced along the m-contiguous surplus row (eq (3.6));
//   store   : lane groups are reduced and c0 + sum is written (eq (3.16)).
#include <cstdlib>
#include <cstring>

#include "kernels_common.h"

namespace hdmr {

namespace {

struct WaveLds {
  double *xs;     // d coordinates
  int32_t *qrow;  // 64 queued rows
  double *qw;     // 64 queued weights
};

__device__ __forceinline__ WaveLds wave_lds(char *smem, int wid, int d) {
  size_t per = ((size_t)d * 8 + 64 * 8 + 64 * 4 + 15) & ~(size_t)15;
  char *base = smem + per * wid;
  WaveLds L;
  L.xs = reinterpret_cast<double *>(base);
  L.qw = reinterpret_cast<double *>(base + (size_t)d * 8);
  L.qrow = reinterpret_cast<int32_t *>(base + (size_t)d * 8 + 64 * 8);
  return L;
}

// Stage one point in LDS; returns true (wave-uniform) if any coordinate is NaN.
__device__ __forceinline__ bool stage_point(const double *__restrict__ X, int64_t p, int d, double *xs, int lane) {
  bool nan_here = false;
  for (int q = lane; q < d; q += WAVE) {
    double v = X[p * d + q];
    xs[q] = v;
    nan_here |= (v != v);
  }
  wave_sync();
  return ballot(nan_here) != 0;
}

// OW lanes per hit (power of two, >= m when m <= 64), OPL outputs per lane.
template <int OW, int OPL>
__global__ __launch_bounds__(256) void k_eval_fp64(ModelView M, const double *__restrict__ X, int64_t n,
                                                   double *__restrict__ Y) {
  extern __shared__ __align__(16) char smem[];
  constexpr int HPI = WAVE / OW;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  const int d = M.d, m = M.m;
  WaveLds L = wave_lds(smem, wid, d);
  const int sub = lane / OW;   // hit slot within one contraction instruction
  const int ol = lane % OW;    // output lane
  const int64_t wave_id = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wid;
  const int64_t nwaves = (int64_t)gridDim.x * WAVES_PER_BLOCK;
  for (int64_t p = wave_id; p < n; p += nwaves) {
    bool is_nan = stage_point(X, p, d, L.xs, lane);
    double acc[OPL];
#pragma unroll
    for (int j = 0; j < OPL; ++j) acc[j] = 0.0;
    // software pipeline over groups of 64 level multi-indices: the directory
    // lookups of group g + 1 are issued before the surplus rows of group g's
    // hits are loaded; the descriptors run one group further ahead
    TupDesc Tn{};
    if (WAVE + lane < M.ntup) Tn = M.tups[WAVE + lane];
    int32_t row = -1;
    double w = 0.0;
    {
      TupDesc T{};
      if (lane < M.ntup) T = M.tups[lane];
      group_lookup(M, L.xs, lane, T, row, w);
    }
    for (int t0 = 0; t0 < M.ntup; t0 += WAVE) {
      // ---- compact hits (ballot + prefix) ----
      const bool hit = row >= 0;
      const uint64_t mask = ballot(hit);
      const int cnt = __popcll(mask);
      if (hit) {
        const int pos = lanes_below(mask);
        L.qrow[pos] = row;
        L.qw[pos] = w;
      }
      wave_sync();
      // ---- next group's lookups ----
      row = -1;
      w = 0.0;
      if (t0 + WAVE < M.ntup) {
        const TupDesc T = Tn;
        if (t0 + 2 * WAVE + lane < M.ntup) Tn = M.tups[t0 + 2 * WAVE + lane];
        group_lookup(M, L.xs, t0 + WAVE + lane < M.ntup ? lane : -1, T, row, w);
      }
      // ---- contract: lanes over outputs, up to HF hits per step with all
      // their row loads in flight; each lane adds its hits in queue order ----
      constexpr int HF = OPL == 1 ? 8 : 4;
      for (int h = sub; h < cnt; h += HF * HPI) {
        int32_t r[HF];
        double ww[HF];
#pragma unroll
        for (int u = 0; u < HF; ++u) {
          const int e = h + u * HPI;
          const int ec = e < cnt ? e : 0;
          r[u] = L.qrow[ec];
          ww[u] = L.qw[ec];
        }
#pragma unroll
        for (int j = 0; j < OPL; ++j) {
          const int o = ol + j * WAVE;
          if (o < m) {
            double a[HF];
#pragma unroll
            for (int u = 0; u < HF; ++u) a[u] = M.alpha[(int64_t)r[u] * M.ms + o];
#pragma unroll
            for (int u = 0; u < HF; ++u)
              if (h + u * HPI < cnt) acc[j] = fma(ww[u], a[u], acc[j]);
          }
        }
      }
      wave_sync();
    }
#pragma unroll
    for (int j = 0; j < OPL; ++j) acc[j] = reduce_groups<OW>(acc[j]);
    if (sub == 0) {
#pragma unroll
      for (int j = 0; j < OPL; ++j) {
        const int o = ol + j * WAVE;
        if (o < m) Y[p * m + o] = is_nan ? __builtin_nan("") : M.c0[o] + acc[j];
      }
    }
    wave_sync();
  }
}

// Gradient: components are walked in order so that the k partial sums of a
// component stay in registers; at the component's end they are added to
// G[p, dim, :] with device atomics (one wave owns the point, so the adds of a
// point are applied in program order).  G must be zero on entry.
template <int OW, int OPL>
__global__ __launch_bounds__(256) void k_eval_grad_fp64(ModelView M, const double *__restrict__ X, int64_t n,
                                                        double *__restrict__ Y, double *__restrict__ G) {
  extern __shared__ __align__(16) char smem[];
  constexpr int HPI = WAVE / OW;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  const int d = M.d, m = M.m;
  // per wave: xs[d], qw[64], qg[64][KMAX], qrow[64]
  size_t per = ((size_t)d * 8 + 64 * 8 * (1 + KMAX) + 64 * 4 + 15) & ~(size_t)15;
  char *base = smem + per * wid;
  double *xs = reinterpret_cast<double *>(base);
  double *qw = reinterpret_cast<double *>(base + (size_t)d * 8);
  double *qg = qw + 64;
  int32_t *qrow = reinterpret_cast<int32_t *>(qg + 64 * KMAX);
  const int sub = lane / OW;
  const int ol = lane % OW;
  const int64_t wave_id = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wid;
  const int64_t nwaves = (int64_t)gridDim.x * WAVES_PER_BLOCK;
  for (int64_t p = wave_id; p < n; p += nwaves) {
    bool is_nan = stage_point(X, p, d, xs, lane);
    double acc[OPL];
#pragma unroll
    for (int j = 0; j < OPL; ++j) acc[j] = 0.0;
    for (int s = 0; s < M.ncomp; ++s) {
      const int tb = M.comp_tup[s], te = M.comp_tup[s + 1];
      if (tb == te) continue;
      const TupDesc T0 = M.tups[tb];
      const int k = T0.k;
      double gacc[KMAX][OPL];
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
#pragma unroll
        for (int j = 0; j < OPL; ++j) gacc[q][j] = 0.0;
      for (int t0 = tb; t0 < te; t0 += WAVE) {
        const int t = t0 + lane;
        int32_t row = -1;
        double w = 0.0, g[KMAX] = {0.0, 0.0, 0.0, 0.0};
        if (t < te) {
          const TupDesc T = M.tups[t];
          double ph[KMAX], dp[KMAX];
          uint32_t slot = 0;
#pragma unroll
          for (int q = 0; q < KMAX; ++q) {
            ph[q] = 1.0;
            dp[q] = 0.0;
            if (q < T.k) {
              uint32_t half, c;
              double tt;
              const double x = xs[T.dims[q]];
              active_cell(x, T.lv[q], half, ph[q], tt, c);
              const double scale = (double)(1u << T.lv[q]);
              // right derivative (left at x = 1); zero outside [0,1]
              dp[q] = (x >= 0.0 && x <= 1.0) ? ((c & 1u) ? -scale : scale) : 0.0;
              slot = (slot << (T.lv[q] - 1)) | half;
            }
          }
          w = T.w;
#pragma unroll
          for (int q = 0; q < KMAX; ++q) w *= ph[q];
          bool any = (w != 0.0);
#pragma unroll
          for (int q = 0; q < KMAX; ++q) {
            if (q < T.k) {
              double gq = T.w * dp[q];
#pragma unroll
              for (int r = 0; r < KMAX; ++r)
                if (r != q) gq *= ph[r];
              g[q] = gq;
              any |= (gq != 0.0);
            }
          }
          if (any) row = lookup_row(T, slot, M.tab);
        }
        const bool hit = row >= 0;
        const uint64_t mask = ballot(hit);
        const int cnt = __popcll(mask);
        if (hit) {
          const int pos = lanes_below(mask);
          qrow[pos] = row;
          qw[pos] = w;
#pragma unroll
          for (int q = 0; q < KMAX; ++q) qg[pos * KMAX + q] = g[q];
        }
        wave_sync();
        for (int h = sub; h < cnt; h += HPI) {
          const int32_t r = qrow[h];
          const double ww = qw[h];
#pragma unroll
          for (int j = 0; j < OPL; ++j) {
            const int o = ol + j * WAVE;
            if (o < m) {
              const double a = M.alpha[(int64_t)r * M.ms + o];
              acc[j] = fma(ww, a, acc[j]);
#pragma unroll
              for (int q = 0; q < KMAX; ++q)
                if (q < k) gacc[q][j] = fma(qg[h * KMAX + q], a, gacc[q][j]);
            }
          }
        }
        wave_sync();
      }
#pragma unroll
      for (int q = 0; q < KMAX; ++q) {
        if (q < k) {
          const int dim = T0.dims[q];
#pragma unroll
          for (int j = 0; j < OPL; ++j) {
            const double v = reduce_groups<OW>(gacc[q][j]);
            const int o = ol + j * WAVE;
            if (sub == 0 && o < m && !is_nan) atomicAdd(&G[(p * d + dim) * m + o], v);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < OPL; ++j) acc[j] = reduce_groups<OW>(acc[j]);
    if (sub == 0) {
#pragma unroll
      for (int j = 0; j < OPL; ++j) {
        const int o = ol + j * WAVE;
        if (o < m && Y) Y[p * m + o] = is_nan ? __builtin_nan("") : M.c0[o] + acc[j];
      }
    }
    if (is_nan) {
      for (int64_t e = lane; e < (int64_t)d * m; e += WAVE) G[p * d * m + e] = __builtin_nan("");
    }
    wave_sync();
  }
}

// Lookup phase only: counts hits (nonzero basis products) and probes.
__global__ __launch_bounds__(256) void k_count_hits(ModelView M, const double *__restrict__ X, int64_t n,
                                                    unsigned long long *__restrict__ counters) {
  extern __shared__ __align__(16) char smem[];
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  const int d = M.d;
  double *xs = reinterpret_cast<double *>(smem) + (size_t)wid * d;
  const int64_t wave_id = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wid;
  const int64_t nwaves = (int64_t)gridDim.x * WAVES_PER_BLOCK;
  unsigned long long hits = 0, probes = 0;
  for (int64_t p = wave_id; p < n; p += nwaves) {
    stage_point(X, p, d, xs, lane);
    for (int t = lane; t < M.ntup; t += WAVE) {
      const TupDesc T = M.tups[t];
      double w = T.w;
      uint32_t slot = 0;
#pragma unroll
      for (int q = 0; q < KMAX; ++q) {
        if (q < T.k) {
          uint32_t half, c;
          double phi, tt;
          active_cell(xs[T.dims[q]], T.lv[q], half, phi, tt, c);
          w *= phi;
          slot = (slot << (T.lv[q] - 1)) | half;
        }
      }
      ++probes;
      if (w != 0.0 && lookup_row(T, slot, M.tab) >= 0) ++hits;
    }
    wave_sync();
  }
  atomicAdd(&counters[0], hits);
  atomicAdd(&counters[1], probes);
}

__global__ void k_fill(double *__restrict__ a, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = v;
}

int grid_for(int64_t n) {
  int64_t blocks = (n + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  return (int)std::min<int64_t>(std::max<int64_t>(blocks, 1), 256 * 16);
}

#define EVAL_DISPATCH(KERNEL, SMEM, ...)                                                       \
  do {                                                                                         \
    const int m_ = M.m;                                                                        \
    dim3 grid_(grid_for(n)), block_(WAVE * WAVES_PER_BLOCK);                                  \
    if (m_ <= 4) hipLaunchKernelGGL((KERNEL<4, 1>), grid_, block_, SMEM, stream, __VA_ARGS__); \
    else if (m_ <= 8) hipLaunchKernelGGL((KERNEL<8, 1>), grid_, block_, SMEM, stream, __VA_ARGS__); \
    else if (m_ <= 16) hipLaunchKernelGGL((KERNEL<16, 1>), grid_, block_, SMEM, stream, __VA_ARGS__); \
    else if (m_ <= 32) hipLaunchKernelGGL((KERNEL<32, 1>), grid_, block_, SMEM, stream, __VA_ARGS__); \
    else if (m_ <= 64) hipLaunchKernelGGL((KERNEL<64, 1>), grid_, block_, SMEM, stream, __VA_ARGS__); \
    else if (m_ <= 128) hipLaunchKernelGGL((KERNEL<64, 2>), grid_, block_, SMEM, stream, __VA_ARGS__); \
    else if (m_ <= 192) hipLaunchKernelGGL((KERNEL<64, 3>), grid_, block_, SMEM, stream, __VA_ARGS__); \
    else hipLaunchKernelGGL((KERNEL<64, 4>), grid_, block_, SMEM, stream, __VA_ARGS__);      \
  } while (0)

// Large batches go through the cell-sorted kernels; small ones (and models
// without grid points) through the single-launch gather kernel.  The
// environment variable HDMR_EVAL_PATH=gather|sorted overrides the choice.
bool use_sorted_path(const hdmr_model *model, int64_t n) {
  if (model->passes.empty()) return false;
  const char *env = std::getenv("HDMR_EVAL_PATH");
  if (env && std::strcmp(env, "gather") == 0) return false;
  if (env && std::strcmp(env, "sorted") == 0) return true;
  return n >= 16384;
}

int check_eval_args(const hdmr_model *model, const double *points, int64_t n, const double *values, int32_t m,
                    bool values_required) {
  if (!model) return fail(HDMR_EINVAL, "null model");
  if (n < 0) return fail(HDMR_EINVAL, "n must be >= 0");
  if (m != model->m) return fail(HDMR_EINVAL, "m does not match the model (" + std::to_string(model->m) + ")");
  if (m > 256) return fail(HDMR_EUNSUPPORTED, "m > 256 is not supported");
  if (n > 0 && (!points || (values_required && !values)))
    return fail(HDMR_EINVAL, "null points or values");
  if (((uintptr_t)points & 7) || ((uintptr_t)values & 7)) return fail(HDMR_EINVAL, "misaligned pointer");
  return HDMR_OK;
}

// hdmr_eval after argument checks: the gather kernel (no workspace) or the
// cell-sorted path with its workspace allocated (ws == NULL) or supplied.
// The environment variable HDMR_SORTED_VARIANT selects another tile shape of
// the cell-sorted path (the variant bits of eval_sorted; diagnostics).
int eval_any(const hdmr_model *model, const double *points, int64_t n, double *values, int precision,
             hipStream_t stream, void *ws, size_t ws_bytes, hipEvent_t *events) {
  if (precision == HDMR_MIXED || use_sorted_path(model, n)) {
    const char *env = std::getenv("HDMR_SORTED_VARIANT");
    const int variant = env ? (std::atoi(env) & 15) : 0;
    return eval_sorted(model, points, n, values, precision, stream, variant, nullptr, ws, ws_bytes, events);
  }
  const ModelView M = model->view();
  const size_t per = ((size_t)M.d * 8 + 64 * 8 + 64 * 4 + 15) & ~(size_t)15;
  const size_t smem = per * WAVES_PER_BLOCK;
  if (smem > 65536) return fail(HDMR_EUNSUPPORTED, "d too large for the LDS staging of points");
  EVAL_DISPATCH(k_eval_fp64, smem, M, points, n, values);
  HDMR_HIP(hipGetLastError());
  return HDMR_OK;
}

}  // namespace

}  // namespace hdmr

using namespace hdmr;

extern "C" {

int hdmr_eval(const hdmr_model *model, const double *points, int64_t n, double *values, int32_t m,
              int32_t precision, hdmr_stream_t stream_) {
  clear_error();
  int rc = check_eval_args(model, points, n, values, m, true);
  if (rc) return rc;
  if (precision != HDMR_PLAIN_FP64 && precision != HDMR_MIXED) return fail(HDMR_EINVAL, "unknown precision");
  if (n == 0) return HDMR_OK;
  if ((rc = set_device_of(model))) return rc;
  return eval_any(model, points, n, values, precision, (hipStream_t)stream_, nullptr, 0, nullptr);
}

int hdmr_eval_noalloc(const hdmr_model *model, const double *points, int64_t n, double *values, int32_t m,
                      int32_t precision, hdmr_stream_t stream_) {
  clear_error();
  int rc = check_eval_args(model, points, n, values, m, true);
  if (rc) return rc;
  if (precision != HDMR_PLAIN_FP64 && precision != HDMR_MIXED) return fail(HDMR_EINVAL, "unknown precision");
  if (n == 0) return HDMR_OK;
  if ((rc = set_device_of(model))) return rc;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  hipEvent_t *events = nullptr;
  if ((rc = noalloc_workspace(model->device, &ws, &ws_bytes, &events))) return rc;
  if (precision == HDMR_MIXED || use_sorted_path(model, n)) {
    size_t need = 0;
    if ((rc = eval_sorted_workspace(model, n, precision, &need))) return rc;
    if (need > ws_bytes)
      return fail(HDMR_EINVAL, "hdmr_eval_noalloc: " + std::to_string(n) + " points of this model need " +
                                   std::to_string(need) + " bytes of workspace; the static workspace holds " +
                                   std::to_string(ws_bytes) + " (use hdmr_eval, or fewer points per call)");
  }
  return eval_any(model, points, n, values, precision, (hipStream_t)stream_, ws, ws_bytes, events);
}

int hdmr_eval_stats(const hdmr_model *model, const double *points, int64_t n, int64_t *hits, int64_t *probes,
                    hdmr_stream_t stream_) {
  clear_error();
  int rc = check_eval_args(model, points, n, nullptr, model ? model->m : 0, false);
  if (rc) return rc;
  if (!hits || !probes) return fail(HDMR_EINVAL, "null output");
  *hits = 0;
  *probes = 0;
  if (n == 0) return HDMR_OK;
  if ((rc = set_device_of(model))) return rc;
  hipStream_t stream = (hipStream_t)stream_;
  const ModelView M = model->view();
  const size_t smem = (size_t)M.d * 8 * WAVES_PER_BLOCK;
  if (smem > 65536) return fail(HDMR_EUNSUPPORTED, "d too large for the LDS staging of points");
  unsigned long long *dc = nullptr, hc[2] = {0, 0};
  HDMR_HIP(dev_malloc((void **)&dc, sizeof(hc)));
  hipError_t e = hipMemsetAsync(dc, 0, sizeof(hc), stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_count_hits, dim3(grid_for(n)), dim3(WAVE * WAVES_PER_BLOCK), smem, stream, M, points, n, dc);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(hc, dc, sizeof(hc), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  (void)hipFree(dc);
  if (e != hipSuccess) return hip_fail(e, "k_count_hits");
  *hits = (int64_t)hc[0];
  *probes = (int64_t)hc[1];
  return HDMR_OK;
}

int hdmr_eval_grad(const hdmr_model *model, const double *points, int64_t n, double *values, double *grad,
                   int32_t m, hdmr_stream_t stream_) {
  clear_error();
  int rc = check_eval_args(model, points, n, values, m, false);
  if (rc) return rc;
  if (n > 0 && !grad) return fail(HDMR_EINVAL, "null grad");
  if ((uintptr_t)grad & 7) return fail(HDMR_EINVAL, "misaligned pointer");
  if (n == 0) return HDMR_OK;
  if ((rc = set_device_of(model))) return rc;
  hipStream_t stream = (hipStream_t)stream_;
  if (use_sorted_path(model, n)) {
    // values are produced alongside; a scratch buffer stands in when not wanted
    double *F = values;
    if (!F) HDMR_HIP(dev_malloc_async((void **)&F, sizeof(double) * (size_t)n * model->m, stream));
    rc = eval_sorted(model, points, n, F, HDMR_PLAIN_FP64, stream, 0, grad);
    if (!values) (void)hipFreeAsync(F, stream);
    return rc;
  }
  const ModelView M = model->view();
  const int64_t total = n * (int64_t)M.d * M.m;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)), dim3(256), 0, stream,
                     grad, total, 0.0);
  const size_t per = ((size_t)M.d * 8 + 64 * 8 * (1 + KMAX) + 64 * 4 + 15) & ~(size_t)15;
  const size_t smem = per * WAVES_PER_BLOCK;
  if (smem > 65536) return fail(HDMR_EUNSUPPORTED, "d too large for the LDS staging of points");
  EVAL_DISPATCH(k_eval_grad_fp64, smem, M, points, n, values, grad);
  HDMR_HIP(hipGetLastError());
  return HDMR_OK;
}

}  // extern "C"
