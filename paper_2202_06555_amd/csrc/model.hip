// Model construction and life cycle: validation of grids (eq (3.3)), the
// per-level-multi-index lookup directory, upload to HBM, export, errors.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>

#include "hdmr_internal.h"

namespace hdmr {

static thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? HDMR_ENOMEM : HDMR_EDEVICE;
}

void clear_error() { g_last_error.clear(); }

namespace {
std::mutex g_inject_mu;
std::string g_inject_val;
int64_t g_inject_count = 0;

bool injected_alloc_failure() {
  const char *v = std::getenv("HDMR_FAIL_ALLOC");
  const std::string s = v ? v : "";
  std::lock_guard<std::mutex> lk(g_inject_mu);
  if (s != g_inject_val) {
    g_inject_val = s;
    g_inject_count = 0;
  }
  if (s.empty()) return false;
  char *end = nullptr;
  const long long k = std::strtoll(s.c_str(), &end, 10);
  if (end == s.c_str() || k < 0) return false;
  return g_inject_count++ == k;
}
}  // namespace

hipError_t dev_malloc(void **p, size_t bytes) {
  if (injected_alloc_failure()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

hipError_t dev_malloc_async(void **p, size_t bytes, hipStream_t s) {
  if (injected_alloc_failure()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMallocAsync(p, bytes, s);
}

int set_device_of(const hdmr_model *model) {
  int cur = -1;
  HDMR_HIP(hipGetDevice(&cur));
  if (cur != model->device) HDMR_HIP(hipSetDevice(model->device));
  keep_pool_memory(model->device);
  return HDMR_OK;
}

// Evaluation workspaces (several GB for large batches) come from the device's
// default stream-ordered pool; keeping freed blocks in the pool (instead of
// returning them at every synchronisation) makes repeated evaluations reuse
// them.  Set once per device.
void keep_pool_memory(int device) {
  static std::mutex mu;
  static std::vector<char> done;
  std::lock_guard<std::mutex> lk(mu);
  if (device < 0) return;
  if ((int)done.size() <= device) done.resize((size_t)device + 1, 0);
  if (done[(size_t)device]) return;
  done[(size_t)device] = 1;
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
    uint64_t threshold = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
  }
}

namespace {

struct RowKey {
  uint32_t lvkey;  // levels packed, first dimension in the high byte
  uint32_t slot;
  int32_t lsum;
  int64_t src;     // source row
};

template <typename T>
int dev_upload(T **dst, const T *src, size_t count, int64_t *bytes) {
  size_t nb = std::max<size_t>(count, 1) * sizeof(T);
  HDMR_HIP(dev_malloc((void **)dst, nb));
  if (count) HDMR_HIP(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  *bytes += (int64_t)nb;
  return HDMR_OK;
}

void free_device(hdmr_model *M) {
  (void)hipFree(M->tups);
  (void)hipFree(M->tab);
  (void)hipFree(M->alpha);
  (void)hipFree(M->alpha32);
  (void)hipFree(M->c0);
  (void)hipFree(M->comp_tup);
  (void)hipFree(M->pass_tups);
  M->pass_tups = nullptr;
  M->tups = nullptr;
  M->tab = nullptr;
  M->alpha = nullptr;
  M->alpha32 = nullptr;
  M->c0 = nullptr;
  M->comp_tup = nullptr;
}

}  // namespace

__global__ void k_to_f32(float *__restrict__ dst, const double *__restrict__ src, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

__global__ void k_gather_rows(double *__restrict__ dst, const double *__restrict__ src, const int64_t *__restrict__ map,
                              int64_t nrows, int32_t m, int32_t ms, int32_t stride, int32_t col) {
  const int64_t total = nrows * ms;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ms;
    const int32_t o = (int32_t)(e - r * ms);
    dst[e] = o < m ? src[map[r] * stride + col + o] : 0.0;
  }
}

int make_model(int32_t d, int32_t m, const double *c0, const std::vector<HostComponent> &hc, hdmr_model **out,
               const DeviceAlphaSource *dsrc) {
  if (d < 1 || d > 32767) return fail(HDMR_EINVAL, "d must be in [1, 32767]");
  if (m < 1) return fail(HDMR_EINVAL, "m must be >= 1");
  auto M = new (std::nothrow) hdmr_model();
  if (!M) return fail(HDMR_ENOMEM, "host allocation failed");
  M->d = d;
  M->m = m;
  M->ms = (m + 1) & ~1;
  const int32_t ms = M->ms;
  M->c0_h.assign(c0, c0 + m);
  int64_t total = 0;
  for (auto &c : hc) total += c.n;
  if (total >= (int64_t)INT32_MAX) {
    delete M;
    return fail(HDMR_EUNSUPPORTED, "more than 2^31-1 rows in one model");
  }
  M->lv_h.assign((size_t)total * KMAX, 0);
  M->ix_h.assign((size_t)total * KMAX, 0);
  std::vector<double> alpha_sorted(dsrc ? 0 : (size_t)total * ms, 0.0);
  std::vector<int64_t> gather(dsrc ? (size_t)total : 0);
  std::vector<int32_t> tab;
  std::vector<int32_t> comp_tup;
  int64_t row0 = 0;
  for (size_t s = 0; s < hc.size(); ++s) {
    const HostComponent &c = hc[s];
    if (c.k < 1 || c.k > KMAX) {
      delete M;
      return fail(HDMR_EUNSUPPORTED, "component " + std::to_string(s) + ": |S| must be in [1, 4]");
    }
    for (int q = 0; q < c.k; ++q) {
      if (c.dims[q] < 0 || c.dims[q] >= d) {
        delete M;
        return fail(HDMR_EINVAL, "component " + std::to_string(s) + ": dimension out of range");
      }
      for (int r = 0; r < q; ++r)
        if (c.dims[r] == c.dims[q]) {
          delete M;
          return fail(HDMR_EINVAL, "component " + std::to_string(s) + ": repeated dimension");
        }
    }
    // validate rows (eq (3.3)) and compute their cell keys
    std::vector<RowKey> keys((size_t)c.n);
    for (int64_t j = 0; j < c.n; ++j) {
      uint32_t lk = 0;
      int32_t ls = 0, sl = 0;
      uint64_t slot = 0;
      for (int q = 0; q < c.k; ++q) {
        int l = c.lv[j * c.k + q];
        uint32_t i = c.ix[j * c.k + q];
        if (l < 1 || l > MAX_LEVEL || (i & 1u) == 0 || (uint64_t)i >= (1ull << l)) {
          delete M;
          return fail(HDMR_EINVAL, "component " + std::to_string(s) + ", row " + std::to_string(j) +
                                       ": level must be in [1,30] and index odd with 0 < i < 2^l");
        }
        lk = (lk << 8) | (uint32_t)l;
        ls += l;
        sl += l - 1;
        slot = (slot << (l - 1)) | ((i - 1) >> 1);
      }
      if (sl > 31) {
        delete M;
        return fail(HDMR_EUNSUPPORTED, "component " + std::to_string(s) + ": sum of (l_q - 1) exceeds 31");
      }
      keys[j] = RowKey{lk, (uint32_t)slot, ls, j};
    }
    std::sort(keys.begin(), keys.end(), [](const RowKey &a, const RowKey &b) {
      if (a.lsum != b.lsum) return a.lsum < b.lsum;
      if (a.lvkey != b.lvkey) return a.lvkey < b.lvkey;
      if (a.slot != b.slot) return a.slot < b.slot;
      return a.src < b.src;
    });
    for (int64_t t = 1; t < c.n; ++t)
      if (keys[t].lvkey == keys[t - 1].lvkey && keys[t].slot == keys[t - 1].slot) {
        delete M;
        return fail(HDMR_EINVAL, "component " + std::to_string(s) + ": duplicate grid point");
      }
    Component comp{};
    comp.k = c.k;
    for (int q = 0; q < KMAX; ++q) comp.dims[q] = q < c.k ? c.dims[q] : 0;
    comp.w = c.w;
    comp.row_begin = row0;
    comp.row_end = row0 + c.n;
    comp.tup_begin = (int32_t)M->tups_h.size();
    comp_tup.push_back(comp.tup_begin);
    for (int64_t t = 0; t < c.n; ++t) {
      int64_t j = keys[t].src, r = row0 + t;
      for (int q = 0; q < c.k; ++q) {
        M->lv_h[r * KMAX + q] = c.lv[j * c.k + q];
        M->ix_h[r * KMAX + q] = c.ix[j * c.k + q];
        M->max_level = std::max<int32_t>(M->max_level, c.lv[j * c.k + q]);
      }
      if (dsrc)
        gather[(size_t)r] = c.src_rows[j];
      else
        std::memcpy(&alpha_sorted[(size_t)r * ms], c.alpha + j * m, sizeof(double) * m);
    }
    // one directory entry per stored level multi-index
    int64_t t0 = 0;
    while (t0 < c.n) {
      int64_t t1 = t0;
      while (t1 < c.n && keys[t1].lvkey == keys[t0].lvkey) ++t1;
      TupDesc T{};
      T.w = c.w;
      T.row_base = (int32_t)(row0 + t0);
      T.comp = (int32_t)s;
      T.k = (uint8_t)c.k;
      T.lsum = (uint8_t)keys[t0].lsum;
      int64_t ncells = 1;
      for (int q = 0; q < c.k; ++q) {
        T.dims[q] = (int16_t)c.dims[q];
        T.lv[q] = (uint8_t)(keys[t0].lvkey >> (8 * (c.k - 1 - q)));
        ncells <<= (T.lv[q] - 1);
      }
      int64_t nr = t1 - t0;
      if (nr == ncells) {
        T.kind = TUP_FULL;
      } else if (ncells <= 4 * nr + 64) {
        T.kind = TUP_DENSE;
        T.aux = (int32_t)tab.size();
        tab.resize(tab.size() + (size_t)ncells, -1);
        for (int64_t t = t0; t < t1; ++t) tab[(size_t)T.aux + keys[t].slot] = (int32_t)(row0 + t);
      } else {
        T.kind = TUP_HASH;
        int64_t cap = 4;
        while (cap < 2 * nr) cap <<= 1;
        if (tab.size() & 1) tab.push_back(0);
        T.aux = (int32_t)tab.size();
        T.mask = (int32_t)(cap - 1);
        tab.resize(tab.size() + 2 * (size_t)cap, 0);
        for (int64_t e = 0; e < cap; ++e) tab[(size_t)T.aux + 2 * e] = (int32_t)HASH_EMPTY;
        for (int64_t t = t0; t < t1; ++t) {
          uint32_t h = slot_hash(keys[t].slot) & (uint32_t)T.mask;
          while ((uint32_t)tab[(size_t)T.aux + 2 * h] != HASH_EMPTY) h = (h + 1) & (uint32_t)T.mask;
          tab[(size_t)T.aux + 2 * h] = (int32_t)keys[t].slot;
          tab[(size_t)T.aux + 2 * h + 1] = (int32_t)(row0 + t);
        }
      }
      if (tab.size() >= (size_t)INT32_MAX) {
        delete M;
        return fail(HDMR_EUNSUPPORTED, "lookup directory exceeds 2^31 entries");
      }
      M->tups_h.push_back(T);
      t0 = t1;
    }
    comp.tup_end = (int32_t)M->tups_h.size();
    M->comps.push_back(comp);
    M->max_k = std::max(M->max_k, c.k);
    row0 += c.n;
  }
  comp_tup.push_back((int32_t)M->tups_h.size());
  M->n_rows = total;
  M->tab_entries = (int64_t)tab.size();
  int rc = HDMR_OK;
  hipError_t ge = hipGetDevice(&M->device);
  if (ge != hipSuccess) {
    delete M;
    return hip_fail(ge, "hipGetDevice");
  }
  if ((rc = dev_upload(&M->tups, M->tups_h.data(), M->tups_h.size(), &M->device_bytes)) ||
      (rc = dev_upload(&M->tab, tab.data(), tab.size(), &M->device_bytes)) ||
      (rc = dsrc ? HDMR_OK : dev_upload(&M->alpha, alpha_sorted.data(), alpha_sorted.size(), &M->device_bytes)) ||
      (rc = dev_upload(&M->c0, M->c0_h.data(), M->c0_h.size(), &M->device_bytes)) ||
      (rc = dev_upload(&M->comp_tup, comp_tup.data(), comp_tup.size(), &M->device_bytes))) {
    free_device(M);
    delete M;
    return rc;
  }
  if (dsrc) {
    int64_t *dmap = nullptr;
    int64_t scratch = 0;
    hipError_t e = dev_malloc((void **)&M->alpha, std::max<size_t>((size_t)total * ms, 1) * sizeof(double));
    if (e == hipSuccess) {
      M->device_bytes += std::max<int64_t>(total * ms, 1) * (int64_t)sizeof(double);
      rc = dev_upload(&dmap, gather.data(), gather.size(), &scratch);
      if (rc == HDMR_OK && total > 0) {
        hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)std::min<int64_t>((total * ms + 255) / 256, 65536)),
                           dim3(256), 0, (hipStream_t)0, M->alpha, dsrc->src, dmap, total, m, ms, dsrc->stride,
                           dsrc->col);
        e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = hip_fail(e, "gather surpluses");
      }
      (void)hipFree(dmap);
    } else {
      rc = hip_fail(e, "dev_malloc(alpha)");
    }
    if (rc) {
      free_device(M);
      delete M;
      return rc;
    }
  }
  {
    // FP32 surpluses for the mixed-precision path (same row order and stride)
    const int64_t count = std::max<int64_t>(total * ms, 1);
    hipError_t e = dev_malloc((void **)&M->alpha32, (size_t)count * sizeof(float));
    if (e == hipSuccess) {
      M->device_bytes += count * (int64_t)sizeof(float);
      hipLaunchKernelGGL(k_to_f32, dim3((unsigned)std::min<int64_t>((count + 255) / 256, 65536)), dim3(256), 0,
                         (hipStream_t)0, M->alpha32, M->alpha, total * ms);
      e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
      free_device(M);
      delete M;
      return hip_fail(e, "FP32 surpluses");
    }
  }
  if ((rc = plan_passes(M))) {
    free_device(M);
    delete M;
    return rc;
  }
  *out = M;
  return HDMR_OK;
}

int plan_passes(hdmr_model *M) {
  // one pass per component of the largest order; lower-order components ride
  // along with the first pass whose key holds their dimensions
  M->passes.clear();
  M->pass_tups_h.clear();
  const int nc = (int)M->comps.size();
  std::vector<int> order(nc);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return M->comps[a].k > M->comps[b].k; });
  std::vector<int> owner(nc, -1);
  std::vector<std::vector<int>> members;
  for (int s : order) {
    const Component &c = M->comps[s];
    if (c.tup_begin == c.tup_end) continue;
    int found = -1;
    for (size_t p = 0; p < M->passes.size() && found < 0; ++p) {
      const Pass &P = M->passes[p];
      if ((int)members[p].size() >= PASS_MAX_COMPS) continue;
      bool sub = true;
      for (int q = 0; q < c.k && sub; ++q) {
        bool in = false;
        for (int r = 0; r < P.k; ++r) in |= (P.dims[r] == c.dims[q]);
        sub = in;
      }
      if (sub) found = (int)p;
    }
    if (found < 0 && c.k == 1) {
      // a one-dimensional component outside every pass so far joins a pass of
      // one other such component (a two-dimensional key), halving their passes
      for (size_t p = 0; p < M->passes.size() && found < 0; ++p) {
        Pass &P = M->passes[p];
        if (P.k != 1 || (int)members[p].size() >= PASS_MAX_COMPS) continue;
        bool single = true;
        for (int s2 : members[p]) single &= M->comps[s2].k == 1;
        if (!single) continue;
        P.dims[1] = c.dims[0];
        P.k = 2;
        found = (int)p;
      }
    }
    if (found < 0) {
      Pass P{};
      P.k = c.k;
      for (int q = 0; q < c.k; ++q) P.dims[q] = c.dims[q];
      M->passes.push_back(P);
      members.emplace_back();
      found = (int)M->passes.size() - 1;
    }
    members[found].push_back(s);
    owner[s] = found;
  }
  for (size_t p = 0; p < M->passes.size(); ++p) {
    Pass &P = M->passes[p];
    int lmax[KMAX] = {0, 0, 0, 0};
    P.tup_begin = (int32_t)M->pass_tups_h.size();
    for (int s : members[p]) {
      const Component &c = M->comps[s];
      for (int t = c.tup_begin; t < c.tup_end; ++t) {
        const TupDesc &T = M->tups_h[t];
        PassTup pt{};
        pt.tup = t;
        for (int q = 0; q < T.k; ++q) {
          int pos = 0;
          while (P.dims[pos] != T.dims[q]) ++pos;
          pt.pos[q] = (uint8_t)pos;
          lmax[pos] = std::max<int>(lmax[pos], T.lv[q]);
        }
        M->pass_tups_h.push_back(pt);
      }
    }
    P.tup_end = (int32_t)M->pass_tups_h.size();
    M->max_pass_tups = std::max(M->max_pass_tups, P.tup_end - P.tup_begin);
    // cells of a pass: one level below the finest stored level per key
    // dimension (a cell of level c lies inside one support of every level
    // <= c + 1, so each level multi-index still has one candidate row per
    // cell), within a 16-bit key
    const int cap = 16 / P.k;
    int shift = 0;
    for (int q = P.k - 1; q >= 0; --q) {
      P.cell_lv[q] = std::max(1, std::min(lmax[q] - 1, cap));
      P.shift[q] = shift;
      shift += P.cell_lv[q];
    }
    P.key_bits = shift;
    // (cell, row) incidences over all cells: along one key dimension a row of
    // level l <= c covers 2^(c - l + 1) of the 2^c cells, a finer row one;
    // a key dimension the tuple lacks contributes all its 2^c cells
    P.list_bound = 0;
    for (int j = P.tup_begin; j < P.tup_end; ++j) {
      const PassTup &pt = M->pass_tups_h[j];
      const TupDesc &T = M->tups_h[pt.tup];
      const Component &c = M->comps[T.comp];
      const int64_t next = pt.tup + 1 < c.tup_end ? (int64_t)M->tups_h[pt.tup + 1].row_base : c.row_end;
      int64_t cover = next - T.row_base;
      bool has[KMAX] = {false, false, false, false};
      for (int q = 0; q < T.k; ++q) {
        const int pos = pt.pos[q], l = T.lv[q], cl = P.cell_lv[pos];
        has[pos] = true;
        if (l <= cl) cover <<= (cl - l + 1);
      }
      for (int q = 0; q < P.k; ++q)
        if (!has[q]) cover <<= P.cell_lv[q];
      P.list_bound += cover;
    }
  }
  int64_t scratch = 0;
  (void)hipFree(M->pass_tups);
  M->pass_tups = nullptr;
  return dev_upload(&M->pass_tups, M->pass_tups_h.data(), M->pass_tups_h.size(), &scratch);
}

}  // namespace hdmr

using namespace hdmr;

extern "C" {

int hdmr_init(int32_t device) {
  clear_error();
  int n = 0;
  HDMR_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(HDMR_EDEVICE, "no such HIP device");
  HDMR_HIP(hipSetDevice(device));
  HDMR_HIP(hipFree(nullptr));
  return noalloc_setup(device);
}

int hdmr_model_from_surpluses(int32_t d, int32_t m, const double *c0, int32_t n_components,
                              const int32_t *comp_offsets, const int32_t *comp_dims,
                              const int64_t *comp_npts, const uint8_t *levels, const uint32_t *indices,
                              const double *surpluses, const double *weights, hdmr_model **out) {
  clear_error();
  if (!out || !c0 || n_components < 0 || (n_components > 0 && (!comp_offsets || !comp_dims || !comp_npts ||
                                                               !levels || !indices || !surpluses || !weights)))
    return fail(HDMR_EINVAL, "hdmr_model_from_surpluses: null argument");
  *out = nullptr;
  std::vector<HostComponent> hc((size_t)n_components);
  int64_t lo = 0, ao = 0;
  for (int32_t s = 0; s < n_components; ++s) {
    int k = comp_offsets[s + 1] - comp_offsets[s];
    if (k < 1 || k > KMAX) return fail(HDMR_EUNSUPPORTED, "component sizes must be in [1, 4]");
    if (comp_npts[s] < 0) return fail(HDMR_EINVAL, "negative point count");
    HostComponent &c = hc[(size_t)s];
    c.k = k;
    for (int q = 0; q < k; ++q) c.dims[q] = comp_dims[comp_offsets[s] + q];
    c.w = weights[s];
    c.n = comp_npts[s];
    c.lv = levels + lo;
    c.ix = indices + lo;
    c.alpha = surpluses + ao;
    lo += c.n * k;
    ao += c.n * m;
  }
  return make_model(d, m, c0, hc, out);
}

int hdmr_get_info(const hdmr_model *model, hdmr_model_info *info) {
  clear_error();
  if (!model || !info) return fail(HDMR_EINVAL, "hdmr_get_info: null argument");
  info->d = model->d;
  info->m = model->m;
  info->n_components = (int32_t)model->comps.size();
  info->n_tuples = (int32_t)model->tups_h.size();
  info->n_rows = model->n_rows;
  info->device_bytes = model->device_bytes;
  info->max_level = model->max_level;
  info->max_k = model->max_k;
  info->n_passes = (int32_t)model->passes.size();
  info->pass_key_dims = 0;
  for (const Pass &P : model->passes) info->pass_key_dims += P.k;
  return HDMR_OK;
}

int hdmr_export_component(const hdmr_model *model, int32_t comp, int64_t *npts, int32_t *k, int32_t *dims,
                          uint8_t *levels, uint32_t *indices, double *surpluses, double *weight) {
  clear_error();
  if (!model || !npts || comp < 0 || comp >= (int32_t)model->comps.size())
    return fail(HDMR_EINVAL, "hdmr_export_component: bad model or component");
  const Component &c = model->comps[(size_t)comp];
  int64_t n = c.row_end - c.row_begin;
  *npts = n;
  if (k) *k = c.k;
  if (dims)
    for (int q = 0; q < c.k; ++q) dims[q] = c.dims[q];
  if (weight) *weight = c.w;
  if (levels || indices)
    for (int64_t j = 0; j < n; ++j)
      for (int q = 0; q < c.k; ++q) {
        if (levels) levels[j * c.k + q] = model->lv_h[(size_t)(c.row_begin + j) * KMAX + q];
        if (indices) indices[j * c.k + q] = model->ix_h[(size_t)(c.row_begin + j) * KMAX + q];
      }
  if (surpluses && n) {
    int rc = set_device_of(model);
    if (rc) return rc;
    HDMR_HIP(hipMemcpy2D(surpluses, sizeof(double) * model->m, model->alpha + c.row_begin * model->ms,
                         sizeof(double) * model->ms, sizeof(double) * model->m, (size_t)n, hipMemcpyDeviceToHost));
  }
  return HDMR_OK;
}

void hdmr_free(hdmr_model *model) {
  if (!model) return;
  int cur = -1;
  if (hipGetDevice(&cur) == hipSuccess && cur != model->device) (void)hipSetDevice(model->device);
  (void)hipDeviceSynchronize();
  batched_forget(model);
  free_device(model);
  if (cur >= 0 && cur != model->device) (void)hipSetDevice(cur);
  delete model;
}

const char *hdmr_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
