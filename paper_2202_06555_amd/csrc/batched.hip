// Batched evaluation of many models (hdmr_eval_batched).
//
// Models of uneven size, dimension and output width are evaluated together:
//   * a persistent multi-model gather kernel takes every model routed to it
//     in one launch: work units of a few points, ordered by estimated cost
//     (heaviest models first), are handed to wavefronts through a device
//     queue counter until the queue is empty;
//   * an autotuner measures, per (model, size bucket of n, precision), the
//     candidate paths on the call's own data -- the persistent gather kernel
//     (plain precision) and the cell-sorted path with five contraction tile
//     shapes (row batch, work-item size, grid) -- and keeps the fastest for
//     later calls;
//   * mixed-precision models always take the cell-sorted path (the gather
//     kernel computes in FP64 only);
//   * the environment variable HDMR_BATCH_PATH=gather|sorted overrides the
//     measured choice (plain precision; mixed always takes the cell-sorted
//     path), for diagnostics such as profiling one path alone;
//   * the persistent launch (queue reset + kernel) is captured once per batch
//     signature into a hipGraph on a private stream and replayed afterwards;
//     models on the cell-sorted path run after it on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <vector>

#include "kernels_common.h"

namespace hdmr {

namespace {

struct BatchItem {
  ModelView M;
  const double *X;
  double *Y;
  int64_t n;
  int64_t unit_begin;  // first work unit of the item
  int32_t upt;         // points per work unit
  int32_t ow;          // lanes per queued hit (power of two >= m, at most 64)
  int32_t opl;         // outputs per lane (m > 64)
  int32_t pad_;
};

constexpr int UNIT_POINTS = 8;

__global__ void k_zero_u64(unsigned long long *c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0ull;
}

// Persistent gather kernel over many models.  A wavefront takes work units
// from the queue; per point it runs the level multi-indices of the unit's
// model across its lanes (active cell, basis product eq (3.1)-(3.2),
// directory lookup), compacts the hits with ballot + prefix into LDS and
// contracts them with lanes over outputs (eq (3.6)); c0 + sum is written
// (eq (3.16)).  Every wave leaves once the queue counter passes the last unit.
// NOPL: the largest outputs-per-lane count of the launch's items (1: every
// model has m <= 64, and the kernel keeps one accumulator per lane).
template <int NOPL>
__global__ __launch_bounds__(256, NOPL == 1 ? 5 : 4) void k_eval_batched(const BatchItem *__restrict__ items, int nitems,
                                                      int64_t total_units, unsigned long long *__restrict__ counter,
                                                      int dmax) {
  extern __shared__ __align__(16) char smem[];
  const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
  const size_t per = ((size_t)dmax * 8 + 64 * 8 + 64 * 4 + 15) & ~(size_t)15;
  char *base = smem + per * wid;
  double *xs = reinterpret_cast<double *>(base);
  double *qw = reinterpret_cast<double *>(base + (size_t)dmax * 8);
  int32_t *qrow = reinterpret_cast<int32_t *>(base + (size_t)dmax * 8 + 64 * 8);
  for (;;) {
    unsigned long long u = 0;
    if (lane == 0) u = atomicAdd(counter, 1ull);
    u = ((unsigned long long)(uint32_t)__shfl((int)(uint32_t)(u >> 32), 0, WAVE) << 32) |
        (unsigned long long)(uint32_t)__shfl((int)(uint32_t)u, 0, WAVE);
    if ((int64_t)u >= total_units) break;
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].unit_begin <= (int64_t)u) lo = mid;
      else hi = mid - 1;
    }
    const BatchItem &I = items[lo];
    const ModelView M = I.M;
    const int d = M.d, m = M.m, OW = I.ow, opl = I.opl;
    const int HPI = WAVE / OW, sub = lane / OW, ol = lane % OW;
    const int64_t p0 = ((int64_t)u - I.unit_begin) * I.upt;
    const int64_t p1 = min(p0 + I.upt, I.n);
    for (int64_t p = p0; p < p1; ++p) {
      bool nan_here = false;
      for (int q = lane; q < d; q += WAVE) {
        const double v = I.X[p * d + q];
        xs[q] = v;
        nan_here |= (v != v);
      }
      wave_sync();
      const bool is_nan = ballot(nan_here) != 0;
      double acc[NOPL];
#pragma unroll
      for (int j = 0; j < NOPL; ++j) acc[j] = 0.0;
      // Software pipeline over groups of 64 level multi-indices: the
      // directory lookups of group g + 1 are issued before the surplus rows
      // of group g's hits are loaded, so both sets of loads are in flight
      // together; the descriptors run one group further ahead.
      TupDesc Tn{};
      if (WAVE + lane < M.ntup) Tn = M.tups[WAVE + lane];
      int32_t row = -1;
      double w = 0.0;
      {
        TupDesc T{};
        if (lane < M.ntup) T = M.tups[lane];
        group_lookup(M, xs, lane, T, row, w);
      }
      for (int t0 = 0; t0 < M.ntup; t0 += WAVE) {
        const bool hit = row >= 0;
        const uint64_t mask = ballot(hit);
        const int cnt = __popcll(mask);
        if (hit) {
          const int pos = lanes_below(mask);
          qrow[pos] = row;
          qw[pos] = w;
        }
        wave_sync();
        row = -1;
        w = 0.0;
        if (t0 + WAVE < M.ntup) {
          const TupDesc T = Tn;
          if (t0 + 2 * WAVE + lane < M.ntup) Tn = M.tups[t0 + 2 * WAVE + lane];
          group_lookup(M, xs, t0 + WAVE + lane < M.ntup ? lane : -1, T, row, w);
        }
        if (NOPL == 1 || opl == 1) {
          // up to HF hits per step, all their row loads in flight together;
          // each lane adds its hits in queue order
          constexpr int HF = 8;
          const bool on = ol < m;
          for (int h = sub; h < cnt; h += HF * HPI) {
            int32_t r[HF];
            double ww[HF], a[HF];
#pragma unroll
            for (int u = 0; u < HF; ++u) {
              const int e = h + u * HPI;
              const int ec = e < cnt ? e : 0;
              r[u] = qrow[ec];
              ww[u] = qw[ec];
            }
#pragma unroll
            for (int u = 0; u < HF; ++u) a[u] = on ? M.alpha[(int64_t)r[u] * M.ms + ol] : 0.0;
#pragma unroll
            for (int u = 0; u < HF; ++u)
              if (h + u * HPI < cnt) acc[0] = fma(ww[u], a[u], acc[0]);
          }
        } else {
          for (int h = sub; h < cnt; h += HPI) {
            const int32_t r = qrow[h];
            const double ww = qw[h];
#pragma unroll
            for (int j = 0; j < NOPL; ++j) {
              const int o = ol + j * WAVE;
              if (j < opl && o < m) acc[j] = fma(ww, M.alpha[(int64_t)r * M.ms + o], acc[j]);
            }
          }
        }
        wave_sync();
      }
#pragma unroll
      for (int j = 0; j < NOPL; ++j)
        for (int off = OW; off < WAVE; off <<= 1) acc[j] += __shfl_xor(acc[j], off, WAVE);
      if (sub == 0) {
#pragma unroll
        for (int j = 0; j < NOPL; ++j) {
          const int o = ol + j * WAVE;
          if (j < opl && o < m) I.Y[p * m + o] = is_nan ? __builtin_nan("") : M.c0[o] + acc[j];
        }
      }
      wave_sync();
    }
  }
}

// ---- host side ------------------------------------------------------------

// Path codes: the gather kernel, or the cell-sorted path with tile shape
// (variant of eval_sorted) code - 1.
enum PathChoice : int32_t { PATH_NONE = -1, PATH_GATHER = 0, PATH_SORTED = 1 };
constexpr int32_t SORTED_SHAPES[] = {0, 1, 2, 4, 6};  // eval_sorted variants the tuner measures

constexpr int64_t TUNE_MIN_POINTS = 16384;  // below this the gather kernel is used untuned
constexpr size_t GRAPH_CACHE_MAX = 32;

struct TuneKey {
  const hdmr_model *model;
  int bucket;
  int precision;
  bool operator<(const TuneKey &o) const {
    if (model != o.model) return model < o.model;
    if (bucket != o.bucket) return bucket < o.bucket;
    return precision < o.precision;
  }
};

struct GraphKey {
  std::vector<const void *> ptrs;  // per item: model, X, Y
  std::vector<int64_t> ns;
  bool operator==(const GraphKey &o) const { return ptrs == o.ptrs && ns == o.ns; }
};

struct GraphEntry {
  GraphKey key;
  std::vector<const hdmr_model *> models;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  BatchItem *items = nullptr;
  unsigned long long *counter = nullptr;
};

std::mutex g_mu;
std::map<TuneKey, int32_t> g_tune;
std::list<GraphEntry> g_graphs;  // most recently used first
hipStream_t g_capture = nullptr;
int g_capture_dev = -1;

void destroy_entry(GraphEntry &e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.graph) (void)hipGraphDestroy(e.graph);
  (void)hipFree(e.items);
  (void)hipFree(e.counter);
  e.exec = nullptr;
  e.graph = nullptr;
  e.items = nullptr;
  e.counter = nullptr;
}

int bucket_of(int64_t n) { return n <= 1 ? 0 : (int)std::floor(std::log2((double)n)); }

BatchItem make_item(const hdmr_model *mdl, const double *X, double *Y, int64_t n) {
  BatchItem I{};
  I.M = mdl->view();
  I.X = X;
  I.Y = Y;
  I.n = n;
  I.upt = UNIT_POINTS;
  int ow = 1;
  while (ow < std::min(mdl->m, WAVE)) ow <<= 1;
  I.ow = ow;
  I.opl = (mdl->m + WAVE - 1) / WAVE;
  return I;
}

double cost_per_point(const hdmr_model *mdl) {
  return (double)mdl->tups_h.size() * (1.0 + (double)mdl->m / WAVE);
}

// Launch the persistent kernel for the given items (already in device memory).
// maxopl: the largest outputs-per-lane count of the items.
int launch_persistent(const BatchItem *d_items, int nitems, int64_t total_units, unsigned long long *counter, int dmax,
                      int maxopl, hipStream_t s) {
  const size_t per = ((size_t)dmax * 8 + 64 * 8 + 64 * 4 + 15) & ~(size_t)15;
  const size_t smem = per * WAVES_PER_BLOCK;
  int dev = 0, cus = 0, per_cu = 0;
  HDMR_HIP(hipGetDevice(&dev));
  HDMR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const bool narrow = maxopl <= 1;
  HDMR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, narrow ? reinterpret_cast<const void *>(k_eval_batched<1>) : reinterpret_cast<const void *>(k_eval_batched<4>),
      WAVE * WAVES_PER_BLOCK, smem));
  const int64_t want = (total_units + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * std::max(per_cu, 1), want));
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, counter);
  if (narrow)
    hipLaunchKernelGGL(k_eval_batched<1>, dim3(blocks), dim3(WAVE * WAVES_PER_BLOCK), smem, s, d_items, nitems,
                       total_units, counter, dmax);
  else
    hipLaunchKernelGGL(k_eval_batched<4>, dim3(blocks), dim3(WAVE * WAVES_PER_BLOCK), smem, s, d_items, nitems,
                       total_units, counter, dmax);
  HDMR_HIP(hipGetLastError());
  return HDMR_OK;
}

// One model through the persistent kernel (the autotuner's gather candidate);
// uses temporary device memory.
int gather_single(const hdmr_model *mdl, const double *X, double *Y, int64_t n, hipStream_t s) {
  BatchItem I = make_item(mdl, X, Y, n);
  I.unit_begin = 0;
  const int64_t units = (n + UNIT_POINTS - 1) / UNIT_POINTS;
  BatchItem *d_item = nullptr;
  unsigned long long *counter = nullptr;
  HDMR_HIP(dev_malloc_async((void **)&d_item, sizeof(BatchItem), s));
  HDMR_HIP(dev_malloc_async((void **)&counter, sizeof(unsigned long long), s));
  HDMR_HIP(hipMemcpyAsync(d_item, &I, sizeof(BatchItem), hipMemcpyHostToDevice, s));
  int rc = launch_persistent(d_item, 1, units, counter, mdl->d, I.opl, s);
  (void)hipFreeAsync(d_item, s);
  (void)hipFreeAsync(counter, s);
  // the host copy of the item must outlive the asynchronous upload
  hipError_t e = hipStreamSynchronize(s);
  if (!rc && e != hipSuccess) rc = hip_fail(e, "batched gather");
  return rc;
}

int run_path(int32_t path, const hdmr_model *mdl, const double *X, double *Y, int64_t n, int precision,
             hipStream_t s) {
  if (path == PATH_GATHER) return gather_single(mdl, X, Y, n, s);
  return eval_sorted(mdl, X, n, Y, precision, s, path - PATH_SORTED);
}

// Measure the candidates on the call's data; the last one run leaves its
// (correct) values in Y.  Returns the fastest.
int autotune(const hdmr_model *mdl, const double *X, double *Y, int64_t n, int precision, hipStream_t s,
             int32_t *best) {
  std::vector<int32_t> cands;
  if (precision == HDMR_PLAIN_FP64) cands.push_back(PATH_GATHER);
  if (!mdl->passes.empty())
    for (int32_t v : SORTED_SHAPES) cands.push_back(PATH_SORTED + v);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HDMR_HIP(hipEventCreate(&e0));
  HDMR_HIP(hipEventCreate(&e1));
  float best_ms = 0.f;
  *best = cands.empty() ? PATH_GATHER : cands[0];
  int rc = HDMR_OK;
  float gather_ms = -1.f, sorted0_ms = -1.f;
  for (size_t c = 0; c < cands.size() && !rc; ++c) {
    // the other tile shapes are measured only while the cell-sorted path is
    // within 2x of the gather kernel (a path that far behind is not tuned)
    if (cands[c] > PATH_SORTED && gather_ms >= 0.f && sorted0_ms > 2.f * gather_ms) break;
    hipError_t e = hipEventRecord(e0, s);
    if (e == hipSuccess) rc = run_path(cands[c], mdl, X, Y, n, precision, s);
    if (!rc && e == hipSuccess) e = hipEventRecord(e1, s);
    if (!rc && e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (!rc && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (!rc && e != hipSuccess) rc = hip_fail(e, "autotune");
    if (!rc && cands[c] == PATH_GATHER) gather_ms = ms;
    if (!rc && cands[c] == PATH_SORTED) sorted0_ms = ms;
    if (!rc && (c == 0 || ms < best_ms)) {
      best_ms = ms;
      *best = cands[c];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

void batched_forget(const hdmr_model *model) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto it = g_tune.begin(); it != g_tune.end();) {
    if (it->first.model == model) it = g_tune.erase(it);
    else ++it;
  }
  for (auto it = g_graphs.begin(); it != g_graphs.end();) {
    if (std::find(it->models.begin(), it->models.end(), model) != it->models.end()) {
      destroy_entry(*it);
      it = g_graphs.erase(it);
    } else {
      ++it;
    }
  }
}

}  // namespace hdmr

using namespace hdmr;

extern "C" int hdmr_eval_batched(const hdmr_model *const *models, const double *const *points, const int64_t *n,
                                 double *const *values, int32_t count, int32_t precision, int32_t *paths,
                                 hdmr_stream_t stream_) {
  clear_error();
  if (count < 0) return fail(HDMR_EINVAL, "count must be >= 0");
  if (count == 0) return HDMR_OK;
  if (!models || !points || !n || !values) return fail(HDMR_EINVAL, "hdmr_eval_batched: null array");
  if (precision != HDMR_PLAIN_FP64 && precision != HDMR_MIXED) return fail(HDMR_EINVAL, "unknown precision");
  int dev = -1;
  int dmax = 1;
  for (int32_t i = 0; i < count; ++i) {
    const hdmr_model *mdl = models[i];
    if (!mdl) return fail(HDMR_EINVAL, "null model in the batch");
    if (n[i] < 0) return fail(HDMR_EINVAL, "n must be >= 0");
    if (n[i] > 0 && (!points[i] || !values[i])) return fail(HDMR_EINVAL, "null points or values");
    if (((uintptr_t)points[i] & 7) || ((uintptr_t)values[i] & 7)) return fail(HDMR_EINVAL, "misaligned pointer");
    if (mdl->m > 256) return fail(HDMR_EUNSUPPORTED, "m > 256 is not supported");
    if (dev < 0) dev = mdl->device;
    if (mdl->device != dev) return fail(HDMR_EINVAL, "all models of a batch must live on one device");
    dmax = std::max(dmax, (int)mdl->d);
  }
  if (((size_t)dmax * 8 + 64 * 8 + 64 * 4 + 15) * WAVES_PER_BLOCK > 65536)
    return fail(HDMR_EUNSUPPORTED, "d too large for the LDS staging of points");
  int rc = set_device_of(models[0]);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream_;
  std::vector<int32_t> choice((size_t)count, PATH_NONE);
  std::vector<char> done((size_t)count, 0);
  int32_t forced = PATH_NONE;
  if (const char *env = std::getenv("HDMR_BATCH_PATH")) {
    if (!std::strcmp(env, "gather")) forced = PATH_GATHER;
    else if (!std::strcmp(env, "sorted")) forced = PATH_SORTED;
  }
  // ---- path choice (measured once per model, size bucket and precision) ----
  for (int32_t i = 0; i < count && !rc; ++i) {
    if (n[i] == 0) {
      done[i] = 1;
      continue;
    }
    if (models[i]->passes.empty() || (n[i] < TUNE_MIN_POINTS && precision == HDMR_PLAIN_FP64)) {
      choice[i] = PATH_GATHER;  // models without grid points: c0 only, exact in any precision
      continue;
    }
    if (n[i] < TUNE_MIN_POINTS) {
      choice[i] = PATH_SORTED;  // mixed precision: the cell-sorted path, default tile shape
      continue;
    }
    if (forced != PATH_NONE) {
      choice[i] = precision == HDMR_MIXED ? PATH_SORTED : forced;
      continue;
    }
    const TuneKey key{models[i], bucket_of(n[i]), precision};
    bool have = false;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        choice[i] = it->second;
        have = true;
      }
    }
    if (!have) {
      int32_t best = PATH_SORTED;
      rc = autotune(models[i], points[i], values[i], n[i], precision, s, &best);
      if (!rc) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tune[key] = best;
        choice[i] = best;
        done[i] = 1;  // the measurement left correct values
      }
    }
  }
  if (rc) return rc;
  // ---- the persistent multi-model launch, through a cached graph ----
  std::vector<int32_t> gi;
  for (int32_t i = 0; i < count; ++i)
    if (!done[i] && choice[i] == PATH_GATHER) gi.push_back(i);
  std::stable_sort(gi.begin(), gi.end(),
                   [&](int32_t a, int32_t b) { return cost_per_point(models[a]) > cost_per_point(models[b]); });
  if (!gi.empty()) {
    GraphKey key;
    for (int32_t i : gi) {
      key.ptrs.push_back(models[i]);
      key.ptrs.push_back(points[i]);
      key.ptrs.push_back(values[i]);
      key.ns.push_back(n[i]);
    }
    key.ns.push_back(precision);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = std::find_if(g_graphs.begin(), g_graphs.end(), [&](const GraphEntry &e) { return e.key == key; });
    if (it == g_graphs.end()) {
      GraphEntry E;
      E.key = key;
      std::vector<BatchItem> host;
      int64_t units = 0;
      int maxopl = 1;
      for (int32_t i : gi) {
        BatchItem I = make_item(models[i], points[i], values[i], n[i]);
        maxopl = std::max(maxopl, (int)I.opl);
        I.unit_begin = units;
        units += (n[i] + UNIT_POINTS - 1) / UNIT_POINTS;
        host.push_back(I);
        E.models.push_back(models[i]);
      }
      hipError_t e = dev_malloc((void **)&E.items, sizeof(BatchItem) * host.size());
      if (e == hipSuccess) e = dev_malloc((void **)&E.counter, sizeof(unsigned long long));
      if (e == hipSuccess)
        e = hipMemcpy(E.items, host.data(), sizeof(BatchItem) * host.size(), hipMemcpyHostToDevice);
      if (e == hipSuccess && (g_capture == nullptr || g_capture_dev != dev)) {
        if (g_capture) (void)hipStreamDestroy(g_capture);
        g_capture = nullptr;
        e = hipStreamCreateWithFlags(&g_capture, hipStreamNonBlocking);
        g_capture_dev = dev;
      }
      if (e == hipSuccess) e = hipStreamBeginCapture(g_capture, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        rc = launch_persistent(E.items, (int)host.size(), units, E.counter, dmax, maxopl, g_capture);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(g_capture, &g);
        E.graph = g;
        if (!rc && e2 != hipSuccess) rc = hip_fail(e2, "graph capture");
        if (!rc) e = hipGraphInstantiate(&E.exec, E.graph, nullptr, nullptr, 0);
      }
      if (!rc && e != hipSuccess) rc = hip_fail(e, "batched graph");
      if (rc) {
        destroy_entry(E);
        return rc;
      }
      if (g_graphs.size() >= GRAPH_CACHE_MAX) {
        (void)hipDeviceSynchronize();  // the evicted graph may still be in flight
        destroy_entry(g_graphs.back());
        g_graphs.pop_back();
      }
      g_graphs.push_front(E);
      it = g_graphs.begin();
    } else if (it != g_graphs.begin()) {
      g_graphs.splice(g_graphs.begin(), g_graphs, it);
      it = g_graphs.begin();
    }
    HDMR_HIP(hipGraphLaunch(it->exec, s));
  }
  // ---- models on the cell-sorted path ----
  for (int32_t i = 0; i < count && !rc; ++i)
    if (!done[i] && choice[i] != PATH_GATHER) rc = run_path(choice[i], models[i], points[i], values[i], n[i], precision, s);
  if (paths)
    for (int32_t i = 0; i < count; ++i) paths[i] = n[i] == 0 ? PATH_NONE : choice[i];
  return rc;
}
