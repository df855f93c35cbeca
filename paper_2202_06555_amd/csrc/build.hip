// asg_build_components: adaptive cut-HDMR build (Alg. 2) with FP64
// hierarchisation and quadrature on the device.
//
// All components advance together by level sum s.  Per step:
//   host   : the new nodes of every component (root first, then admitted
//            children), the rows x = xbar \ x_v they need (deduplicated over
//            nodes, components and steps), one call of f, and per node the cut
//            value g_S = f(xbar \ x_S) and the component value
//            u_S = sum_v (-1)^{|S|-|v|} f(xbar \ x_v) (eq (2.2.6)) taken as
//            nested differences over the dimensions of S;
//   device : k_hierarchize_fp64 -- alpha = y - (interpolant of the rows of
//            smaller level sum at the node), for g and u together (2m
//            columns), and the eq (3.8) test max_o |alpha^g_o| > eps_gamma;
//   host   : the new level multi-indices join the lookup directory;
//   device : k_refine -- the children (l + e_q, 2 i_q -+ 1) of accepted nodes
//            are admitted by the parent rule (Sec. 3.1 exclusion), each once,
//            and packed for the next step.
// With the Alg. 2 criteria (eps_eta or eps_rho > 0) the expansion orders are
// built in turn: the candidates of order k (index sets of size k that contain
// no rejected set of Z) are grown as above, k_quadrature_rows forms the
// quadrature (eq (3.7)) of every candidate's component interpolant on the
// device, and the host applies the active-dimension test (eq (3.19)) and the
// expansion test (eq (3.18)) to those m-vectors.
// At the end the surpluses of u_S (form 0) or of g_S with the eq (4.2)
// weights (form 1) of the kept components are gathered into a regular model.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <cstring>
#include <thread>
#include <unordered_map>

#include "kernels_common.h"

namespace hdmr {

namespace {

struct NodeDev {
  int32_t comp;
  int32_t row;      // build row receiving the surpluses
  uint8_t lv[KMAX];
  uint32_t ix[KMAX];
};

// One wave per new node: evaluate the component's existing interpolant (all
// rows of smaller level sum) at the node, subtract from the nodal values.
template <int OPL>
__global__ __launch_bounds__(256) void k_hierarchize_fp64(const TupDesc *__restrict__ tups,
                                                          const int32_t *__restrict__ tab, double *__restrict__ alpha,
                                                          int32_t M2, int32_t m, const int32_t *__restrict__ ct_off,
                                                          const int32_t *__restrict__ ct_ids,
                                                          const NodeDev *__restrict__ nodes, int64_t nnodes,
                                                          const double *__restrict__ y, double eps,
                                                          uint8_t *__restrict__ accepted) {
  __shared__ int32_t qrow_s[WAVES_PER_BLOCK][WAVE];
  __shared__ double qw_s[WAVES_PER_BLOCK][WAVE];
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  int32_t *qrow = qrow_s[wid];
  double *qw = qw_s[wid];
  const int64_t wave_id = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wid;
  const int64_t nwaves = (int64_t)gridDim.x * WAVES_PER_BLOCK;
  for (int64_t j = wave_id; j < nnodes; j += nwaves) {
    const NodeDev nd = nodes[j];
    double xs[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) xs[q] = (double)nd.ix[q] / (double)(1u << (nd.lv[q] ? nd.lv[q] : 1));
    double acc[OPL];
#pragma unroll
    for (int u = 0; u < OPL; ++u) acc[u] = 0.0;
    const int tb = ct_off[nd.comp], te = ct_off[nd.comp + 1];
    for (int t0 = tb; t0 < te; t0 += WAVE) {
      const int t = t0 + lane;
      int32_t row = -1;
      double w = 0.0;
      if (t < te) {
        const TupDesc T = tups[ct_ids[t]];
        w = 1.0;
        uint32_t slot = 0;
#pragma unroll
        for (int q = 0; q < KMAX; ++q) {
          if (q < T.k) {
            uint32_t half, c;
            double phi, tt;
            active_cell(xs[q], T.lv[q], half, phi, tt, c);
            w *= phi;
            slot = (slot << (T.lv[q] - 1)) | half;
          }
        }
        if (w != 0.0) row = lookup_row(T, slot, tab);
      }
      const bool hit = row >= 0;
      const uint64_t mask = ballot(hit);
      const int cnt = __popcll(mask);
      if (hit) {
        const int pos = lanes_below(mask);
        qrow[pos] = row;
        qw[pos] = w;
      }
      wave_sync();
      for (int h = 0; h < cnt; ++h) {
        const int32_t r = qrow[h];
        const double ww = qw[h];
#pragma unroll
        for (int u = 0; u < OPL; ++u) {
          const int o = lane + u * WAVE;
          if (o < M2) acc[u] = fma(ww, alpha[(int64_t)r * M2 + o], acc[u]);
        }
      }
      wave_sync();
    }
    double gmax = 0.0;
    bool gnan = false;
#pragma unroll
    for (int u = 0; u < OPL; ++u) {
      const int o = lane + u * WAVE;
      if (o < M2) {
        const double a = y[j * M2 + o] - acc[u];
        alpha[(int64_t)nd.row * M2 + o] = a;
        if (o < m) {
          gmax = fmax(gmax, fabs(a));
          gnan |= (a != a);
        }
      }
    }
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) gmax = fmax(gmax, __shfl_xor(gmax, off, WAVE));
    gnan = ballot(gnan) != 0;
    if (lane == 0) accepted[j] = (eps < 0.0) ? 1 : ((!gnan && gmax > eps) ? 1 : 0);
  }
}

// Quadrature of eq (3.7) for a set of components: q[c * m + o] = sum over the
// listed rows r of component c (row[off[c] .. off[c+1])) of wt[r] *
// A[row[r] * lda + col + o], wt = 2^-|l|_1 the integral of the row's tensor
// basis function.  One workgroup per component; the four waves take every
// fourth row and their partial sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_quadrature_rows(const double *__restrict__ A, int lda, int col, int m,
                                                         const int64_t *__restrict__ row,
                                                         const double *__restrict__ wt,
                                                         const int64_t *__restrict__ off, double *__restrict__ q) {
  __shared__ double part[WAVES_PER_BLOCK][WAVE];
  const int c = blockIdx.x, lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  for (int o0 = 0; o0 < m; o0 += WAVE) {
    const int o = o0 + lane;
    double sum = 0.0;
    if (o < m)
      for (int64_t r = off[c] + w; r < off[c + 1]; r += WAVES_PER_BLOCK)
        sum = fma(wt[r], A[row[r] * lda + col + o], sum);
    part[w][lane] = sum;
    __syncthreads();
    if (w == 0 && o < m) q[(int64_t)c * m + o] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    __syncthreads();
  }
}

// A child admitted for the next step, as k_refine hands it back.
struct ChildDev {
  int32_t comp;
  uint8_t lv[KMAX];
  uint32_t ix[KMAX];
};

// Order of a node among the nodes of one step: (component, the levels as
// 8-bit digits, the cell slot -- the bits (i_q - 1) / 2 of every dimension in
// turn, l_q - 1 bits each).  The host sorts each step's nodes by this key;
// with at most 31 slot bits no two nodes share it.
__device__ __forceinline__ void node_order(const uint8_t *lv, const uint32_t *ix, uint32_t &lk, uint32_t &sl) {
  lk = 0;
  sl = 0;
#pragma unroll
  for (int q = 0; q < KMAX; ++q)
    if (lv[q]) {
      lk = (lk << 8) | lv[q];
      sl = (sl << (lv[q] - 1)) | ((ix[q] - 1) >> 1);
    }
}

// Position of the node (comp, lk, sl) among the step's n nodes, or -1.
__device__ int64_t find_node(const NodeDev *__restrict__ nodes, int64_t n, int32_t comp, uint32_t lk, uint32_t sl) {
  int64_t lo = 0, hi = n;  // first node whose key is not below the target
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const NodeDev v = nodes[mid];
    uint32_t vl, vs;
    node_order(v.lv, v.ix, vl, vs);
    const bool below = v.comp != comp ? v.comp < comp : (vl != lk ? vl < lk : vs < sl);
    if (below) lo = mid + 1;
    else hi = mid;
  }
  if (lo == n) return -1;
  const NodeDev v = nodes[lo];
  uint32_t vl, vs;
  node_order(v.lv, v.ix, vl, vs);
  return (v.comp == comp && vl == lk && vs == sl) ? lo : -1;
}

// The Sec. 3.1 refinement of one step on the device.  One thread per
// candidate t = (node j, dimension q, side): the child (l + e_q, 2 i_q -+ 1)
// of node j, considered when j was accepted (eq (3.8)), q < |S| and the level
// limit allows it.  Its parents -- the child with one level lowered, in each
// dimension whose level exceeds 1 -- have the step's level sum, so they are
// all among the step's nodes, found by binary search.  Rule 0 admits the child
// when every parent is accepted, rule 1 when one is (node j itself is one).
// A child with several parents is emitted once: under rule 0 by its parent in
// the lowest dimension with a parent, under rule 1 by its accepted parent in
// the lowest such dimension.  Emitted children are packed into
// out[0 .. *count) with one ballot and one atomic per wave; their order varies
// from run to run, and the next step sorts them.
__global__ __launch_bounds__(256) void k_refine(const NodeDev *__restrict__ nodes,
                                                const uint8_t *__restrict__ accepted, int64_t n, int max_level,
                                                int level_rule, int refine_rule, ChildDev *__restrict__ out,
                                                uint32_t *__restrict__ count) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t ncand = n * (2 * KMAX);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // the lanes of a wave share t0, so they leave the loop together
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(WAVE - 1)); t0 < ncand; t0 += stride) {
    const int64_t t = t0 + lane;
    bool emit = false;
    ChildDev ch{};
    if (t < ncand && accepted[t / (2 * KMAX)]) {
      const int64_t j = t / (2 * KMAX);
      const int q = (int)((t >> 1) & (KMAX - 1));
      const NodeDev v = nodes[j];
      int k = 0, ls = 0;
#pragma unroll
      for (int r = 0; r < KMAX; ++r)
        if (v.lv[r]) {
          ++k;
          ls += v.lv[r];
        }
      bool ok = q < k && (level_rule == 1 ? ls + 1 <= max_level + k - 1 : v.lv[q] + 1 <= max_level);
      if (ok) {
        ch.comp = v.comp;
#pragma unroll
        for (int r = 0; r < KMAX; ++r) {
          ch.lv[r] = v.lv[r];
          ch.ix[r] = v.ix[r];
        }
        ch.lv[q] = (uint8_t)(ch.lv[q] + 1);
        ch.ix[q] = (t & 1) ? 2 * ch.ix[q] + 1 : 2 * ch.ix[q] - 1;
        // rule 0: only the lowest dimension with a parent emits, and every
        // parent above it must be accepted; rule 1: emit unless a lower
        // dimension has an accepted parent
        for (int p = 0; p < k && ok; ++p) {
          if (p == q || ch.lv[p] <= 1) continue;
          if (refine_rule == 0 && p < q) {
            ok = false;
            break;
          }
          if (refine_rule == 1 && p > q) break;
          uint8_t plv[KMAX];
          uint32_t pix[KMAX];
#pragma unroll
          for (int r = 0; r < KMAX; ++r) {
            plv[r] = ch.lv[r];
            pix[r] = ch.ix[r];
          }
          plv[p] = (uint8_t)(plv[p] - 1);
          const uint32_t a = (pix[p] - 1) >> 1, b = (pix[p] + 1) >> 1;
          pix[p] = (a & 1u) ? a : b;
          uint32_t lk, sl;
          node_order(plv, pix, lk, sl);
          const int64_t pj = find_node(nodes, n, v.comp, lk, sl);
          const bool pacc = pj >= 0 && accepted[pj];
          if (refine_rule == 0 ? !pacc : pacc) ok = false;
        }
        emit = ok;
      }
    }
    const uint64_t mask = ballot(emit);
    if (mask) {
      const int leader = __ffsll((long long)mask) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(mask));
      base = (uint32_t)__shfl((int)base, leader, WAVE);
      if (emit) out[base + lanes_below(mask)] = ch;
    }
  }
}

struct NodeKey {
  std::array<uint8_t, KMAX> l;
  std::array<uint32_t, KMAX> i;
  bool operator==(const NodeKey &o) const { return l == o.l && i == o.i; }
};
struct NodeKeyHash {
  size_t operator()(const NodeKey &k) const {
    uint64_t h = 1469598103934665603ULL;
    for (int q = 0; q < KMAX; ++q) {
      h ^= (uint64_t)k.l[q] * 0x9E3779B97F4A7C15ULL + k.i[q];
      h *= 1099511628211ULL;
      h ^= h >> 31;
    }
    return (size_t)h;
  }
};

// Key of a row xbar \ x_v: the (dimension, value) pairs that differ from xbar.
struct RowKey {
  int32_t n;
  std::array<int32_t, KMAX> dim;
  std::array<uint64_t, KMAX> bits;
  bool operator==(const RowKey &o) const {
    if (n != o.n) return false;
    for (int q = 0; q < n; ++q)
      if (dim[q] != o.dim[q] || bits[q] != o.bits[q]) return false;
    return true;
  }
};
struct RowKeyHash {
  size_t operator()(const RowKey &k) const {
    uint64_t h = 0x12345678ULL + (uint64_t)k.n;
    for (int q = 0; q < k.n; ++q) {
      h ^= (uint64_t)k.dim[q] * 0x9E3779B97F4A7C15ULL;
      h *= 1099511628211ULL;
      h ^= k.bits[q] + (h << 6) + (h >> 2);
    }
    return (size_t)h;
  }
};

struct CompState {
  int32_t k;
  int32_t dims[KMAX];
  std::unordered_map<NodeKey, int32_t, NodeKeyHash> index;  // node -> local row
  std::vector<uint8_t> acc;                                   // per local row
  std::vector<uint8_t> lv;                                    // local rows x k
  std::vector<uint32_t> ix;
  std::vector<int64_t> build_row;                             // local row -> build row
  std::vector<int32_t> tuples;                                // build tuple ids
  std::vector<NodeKey> pending;                               // nodes of the next step
};

// f(begin, end) over [0, n) split into contiguous ranges, one per host
// thread (at most 16; one range when n is small).  Every range's work must be
// independent of the others'.
template <typename F>
void parallel_ranges(int64_t n, int64_t grain, F f) {
  const int64_t hw = std::max<int64_t>(1, std::min<int64_t>(16, (int64_t)std::thread::hardware_concurrency()));
  const int64_t T = std::max<int64_t>(1, std::min<int64_t>(hw, n / std::max<int64_t>(grain, 1)));
  if (T <= 1) {
    f((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve((size_t)T);
  for (int64_t i = 0; i < T; ++i) th.emplace_back([&f, n, T, i]() { f(n * i / T, n * (i + 1) / T); });
  for (auto &x : th) x.join();
}

template <typename T>
int grow_device(T **ptr, int64_t *cap, int64_t need, int64_t used) {
  if (need <= *cap) return HDMR_OK;
  int64_t nc = std::max<int64_t>(*cap * 2, 1024);
  while (nc < need) nc *= 2;
  T *np = nullptr;
  HDMR_HIP(dev_malloc((void **)&np, (size_t)nc * sizeof(T)));
  if (*ptr && used > 0) HDMR_HIP(hipMemcpy(np, *ptr, (size_t)used * sizeof(T), hipMemcpyDeviceToDevice));
  if (*ptr) HDMR_HIP(hipFree(*ptr));
  *ptr = np;
  *cap = nc;
  return HDMR_OK;
}

inline uint64_t dbits(double v) {
  uint64_t b;
  std::memcpy(&b, &v, 8);
  return b;
}

struct DeviceBuffers {
  TupDesc *tups = nullptr;
  int32_t *tab = nullptr;
  double *alpha = nullptr;
  int64_t tups_cap = 0, tab_cap = 0, alpha_cap = 0;
  ~DeviceBuffers() {
    (void)hipFree(tups);
    (void)hipFree(tab);
    (void)hipFree(alpha);
  }
};

// Wall time of the build's phases, printed to stderr at the end of a build
// when the environment variable HDMR_BUILD_PROFILE is set (diagnostics).
struct PhaseClock {
  enum { NODES, ROWS, CALL, NODAL, HIER, DIRECTORY, CHILDREN, QUAD, ASSEMBLE, NPHASE };
  double sec[NPHASE] = {};
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  void lap(int phase) {
    const auto t1 = std::chrono::steady_clock::now();
    sec[phase] += std::chrono::duration<double>(t1 - t0).count();
    t0 = t1;
  }
  void report(int64_t rows, int64_t fcalls) const {
    if (!std::getenv("HDMR_BUILD_PROFILE")) return;
    static const char *names[NPHASE] = {"nodes",     "row keys", "f calls",  "nodal values", "hierarchise",
                                        "directory", "children", "quadrature", "assemble"};
    double total = 0.0;
    for (double s : sec) total += s;
    std::fprintf(stderr, "[hdmr build] %lld grid rows, %lld f rows, %.3f s:", (long long)rows, (long long)fcalls,
                 total);
    for (int i = 0; i < NPHASE; ++i) std::fprintf(stderr, " %s %.3f", names[i], sec[i]);
    std::fprintf(stderr, "\n");
  }
};

}  // namespace

}  // namespace hdmr

using namespace hdmr;

extern "C" int asg_build_components(const asg_build_params *P, hdmr_fn f, void *user, hdmr_model **out) {
  clear_error();
  if (!P || !f || !out || !P->anchor) return fail(HDMR_EINVAL, "asg_build_components: null argument");
  *out = nullptr;
  const int d = P->d, m = P->m, M2 = 2 * m;
  if (d < 1 || d > 32767 || m < 1 || m > 256) return fail(HDMR_EINVAL, "d must be in [1,32767] and m in [1,256]");
  if (P->max_level < 1 || P->max_level > MAX_LEVEL) return fail(HDMR_EINVAL, "max_level must be in [1,30]");
  if (P->level_rule != 0 && P->level_rule != 1) return fail(HDMR_EINVAL, "level_rule must be 0 or 1");
  if (P->refine_rule != 0 && P->refine_rule != 1) return fail(HDMR_EINVAL, "refine_rule must be 0 or 1");
  if (P->form != 0 && P->form != 1) return fail(HDMR_EINVAL, "form must be 0 or 1");
  const bool criteria = P->eps_eta > 0.0 || P->eps_rho > 0.0;
  // HDMR_REFINE=host admits the children on the host instead of with k_refine
  // (diagnostics: the grids are the same)
  const char *refine_env = std::getenv("HDMR_REFINE");
  const bool host_refine = refine_env && std::strcmp(refine_env, "host") == 0;
  if (!(P->eps_eta == P->eps_eta) || !(P->eps_rho == P->eps_rho)) return fail(HDMR_EINVAL, "eps_eta / eps_rho NaN");
  // ---- index sets requested (all of them, or the candidates of Alg. 2) ----
  std::vector<CompState> all;
  if (P->n_components > 0) {
    if (!P->comp_offsets || !P->comp_dims) return fail(HDMR_EINVAL, "null component list");
    for (int s = 0; s < P->n_components; ++s) {
      CompState c;
      c.k = P->comp_offsets[s + 1] - P->comp_offsets[s];
      if (c.k < 1 || c.k > KMAX) return fail(HDMR_EUNSUPPORTED, "component sizes must be in [1,4]");
      for (int q = 0; q < c.k; ++q) {
        c.dims[q] = P->comp_dims[P->comp_offsets[s] + q];
        if (c.dims[q] < 0 || c.dims[q] >= d || (q && c.dims[q] <= c.dims[q - 1]))
          return fail(HDMR_EINVAL, "component dimensions must be strictly increasing and < d");
      }
      all.push_back(std::move(c));
    }
  } else {
    if (P->max_order < 1 || P->max_order > KMAX) return fail(HDMR_EUNSUPPORTED, "max_order must be in [1,4]");
    for (int k = 1; k <= P->max_order; ++k) {
      std::array<int32_t, KMAX> v{};
      for (int q = 0; q < k; ++q) v[q] = q;
      if (k > d) break;
      for (;;) {
        CompState c;
        c.k = k;
        for (int q = 0; q < k; ++q) c.dims[q] = v[q];
        all.push_back(std::move(c));
        int q = k - 1;
        while (q >= 0 && v[q] == d - k + q) --q;
        if (q < 0) break;
        ++v[q];
        for (int r = q + 1; r < k; ++r) v[r] = v[r - 1] + 1;
      }
    }
  }
  std::vector<double> anchor(P->anchor, P->anchor + d);
  auto add_root = [](CompState &c) {
    NodeKey root{};
    for (int q = 0; q < c.k; ++q) {
      root.l[q] = 1;
      root.i[q] = 1;
    }
    c.pending.push_back(root);
  };
  std::vector<CompState> C;  // components grown so far, in build order
  // ---- row cache for f(xbar \ x_v) with |v| < |S| ----
  std::unordered_map<RowKey, int64_t, RowKeyHash> cache;
  std::vector<double> cache_val;
  DeviceBuffers D;
  std::vector<TupDesc> h_tups;
  int64_t tab_used = 0, rows_used = 0;
  int32_t lsum_top = P->level_rule == 1 ? P->max_level + KMAX - 1 : P->max_level * KMAX;
  PhaseClock clk;
  int64_t f_rows = 0;
  // grows every component of C that has pending nodes (new roots) to the end
  auto run_steps = [&]() -> int {
  const int ncomp = (int)C.size();
  for (int32_t step = 1; step <= lsum_top; ++step) {
    // ---- collect this step's nodes ----
    struct NewNode {
      int32_t comp;
      NodeKey key;
      uint32_t lvkey, slot;
    };
    std::vector<NewNode> nn;
    for (int s = 0; s < ncomp; ++s) {
      CompState &c = C[s];
      if (c.pending.empty()) continue;
      int32_t ls0 = 0;
      for (int q = 0; q < c.k; ++q) ls0 += c.pending[0].l[q];
      if (ls0 != step) continue;
      if (ls0 - c.k > 31) return fail(HDMR_EUNSUPPORTED, "a grid point's sum of (l_q - 1) exceeds 31");
      for (const NodeKey &key : c.pending) {
        uint32_t lk = 0, sl = 0;
        for (int q = 0; q < c.k; ++q) {
          lk = (lk << 8) | key.l[q];
          sl = (sl << (key.l[q] - 1)) | ((key.i[q] - 1) >> 1);
        }
        nn.push_back(NewNode{s, key, lk, sl});
      }
      c.pending.clear();
    }
    if (nn.empty()) {
      bool any = false;
      for (auto &c : C) any |= !c.pending.empty();
      if (!any) break;
      continue;
    }
    std::stable_sort(nn.begin(), nn.end(), [](const NewNode &a, const NewNode &b) {
      if (a.comp != b.comp) return a.comp < b.comp;
      if (a.lvkey != b.lvkey) return a.lvkey < b.lvkey;
      return a.slot < b.slot;
    });
    const int64_t N = (int64_t)nn.size();
    clk.lap(PhaseClock::NODES);
    // ---- rows to evaluate ----
    std::vector<int64_t> ref((size_t)N << KMAX, -1);   // per node and subset: cache row or -(fresh+2)
    std::vector<RowKey> fresh_keys;
    std::vector<RowKey> new_cache_keys;
    for (int64_t j = 0; j < N; ++j) {
      const CompState &c = C[nn[j].comp];
      double xs[KMAX];
      for (int q = 0; q < c.k; ++q) xs[q] = std::ldexp((double)nn[j].key.i[q], -(int)nn[j].key.l[q]);
      const int nsub = 1 << c.k;
      for (int v = 0; v < nsub; ++v) {
        RowKey rk{};
        for (int q = 0; q < c.k; ++q)
          if ((v >> q) & 1)
            if (!(xs[q] == anchor[c.dims[q]])) {
              rk.dim[rk.n] = c.dims[q];
              rk.bits[rk.n] = dbits(xs[q]);
              ++rk.n;
            }
        if (v == nsub - 1 && rk.n == c.k) {
          ref[(size_t)(j << KMAX) + v] = -(int64_t)fresh_keys.size() - 2;
          fresh_keys.push_back(rk);
          continue;
        }
        auto it = cache.find(rk);
        if (it == cache.end()) {
          int64_t id = (int64_t)(cache_val.size() / m) + (int64_t)new_cache_keys.size();
          it = cache.emplace(rk, id).first;
          new_cache_keys.push_back(rk);
        }
        ref[(size_t)(j << KMAX) + v] = it->second;
      }
    }
    // ---- one call of f for every new row ----
    const int64_t nfresh = (int64_t)fresh_keys.size(), ncache_new = (int64_t)new_cache_keys.size();
    clk.lap(PhaseClock::ROWS);
    const int64_t nrows_f = nfresh + ncache_new;
    std::vector<double> X((size_t)nrows_f * d), Y((size_t)nrows_f * m);
    for (int64_t r = 0; r < nrows_f; ++r) {
      const RowKey &rk = r < ncache_new ? new_cache_keys[r] : fresh_keys[r - ncache_new];
      double *row = &X[(size_t)r * d];
      std::memcpy(row, anchor.data(), sizeof(double) * d);
      for (int q = 0; q < rk.n; ++q) std::memcpy(&row[rk.dim[q]], &rk.bits[q], 8);
    }
    if (nrows_f > 0 && f(X.data(), nrows_f, d, Y.data(), m, user) != 0)
      return fail(HDMR_ECALLBACK, "the user function returned an error");
    cache_val.insert(cache_val.end(), Y.begin(), Y.begin() + (size_t)ncache_new * m);
    f_rows += nrows_f;
    clk.lap(PhaseClock::CALL);
    // ---- nodal values: g = f(xbar \ x_S), u = nested differences ----
    std::vector<double> yv((size_t)N * M2);
    parallel_ranges(N, 4096, [&](int64_t j0, int64_t j1) {
      std::vector<double> buf((size_t)m << KMAX);
      for (int64_t j = j0; j < j1; ++j) {
        const CompState &c = C[nn[j].comp];
        const int nsub = 1 << c.k;
        for (int v = 0; v < nsub; ++v) {
          const int64_t r = ref[(size_t)(j << KMAX) + v];
          const double *src = r >= 0 ? &cache_val[(size_t)r * m] : &Y[(size_t)(ncache_new + (-r - 2)) * m];
          std::memcpy(&buf[(size_t)v * m], src, sizeof(double) * m);
        }
        for (int o = 0; o < m; ++o) yv[(size_t)j * M2 + o] = buf[(size_t)(nsub - 1) * m + o];
        for (int q = 0; q < c.k; ++q)
          for (int v = 0; v < nsub; ++v)
            if ((v >> q) & 1)
              for (int o = 0; o < m; ++o) buf[(size_t)v * m + o] -= buf[(size_t)(v ^ (1 << q)) * m + o];
        for (int o = 0; o < m; ++o) yv[(size_t)j * M2 + m + o] = buf[(size_t)(nsub - 1) * m + o];
      }
    });
    clk.lap(PhaseClock::NODAL);
    // ---- device: hierarchise against the existing directory ----
    std::vector<NodeDev> nd((size_t)N);
    for (int64_t j = 0; j < N; ++j) {
      nd[j].comp = nn[j].comp;
      nd[j].row = (int32_t)(rows_used + j);
      for (int q = 0; q < KMAX; ++q) {
        nd[j].lv[q] = nn[j].key.l[q];
        nd[j].ix[q] = nn[j].key.i[q];
      }
    }
    std::vector<int32_t> ct_off((size_t)ncomp + 1, 0), ct_ids;
    for (int s = 0; s < ncomp; ++s) {
      ct_off[s] = (int32_t)ct_ids.size();
      ct_ids.insert(ct_ids.end(), C[s].tuples.begin(), C[s].tuples.end());
    }
    ct_off[ncomp] = (int32_t)ct_ids.size();
    if (rows_used + N >= (int64_t)INT32_MAX) return fail(HDMR_EUNSUPPORTED, "more than 2^31-1 grid points");
    int rc = grow_device(&D.alpha, &D.alpha_cap, (rows_used + N) * M2, rows_used * M2);
    if (rc) return rc;
    // the step's device buffers; what k_refine needs lives to the end of the step
    struct StepBuffers {
      NodeDev *nodes = nullptr;
      double *y = nullptr;
      int32_t *ctoff = nullptr, *ctids = nullptr;
      uint8_t *acc = nullptr;
      ChildDev *kids = nullptr;
      uint32_t *nkids = nullptr;
      void free_hier() {
        (void)hipFree(y);
        (void)hipFree(ctoff);
        (void)hipFree(ctids);
        y = nullptr;
        ctoff = ctids = nullptr;
      }
      ~StepBuffers() {
        free_hier();
        (void)hipFree(nodes);
        (void)hipFree(acc);
        (void)hipFree(kids);
        (void)hipFree(nkids);
      }
    } SB;
    std::vector<uint8_t> acc((size_t)N);
    hipError_t e = hipSuccess;
    if ((e = dev_malloc((void **)&SB.nodes, sizeof(NodeDev) * N)) != hipSuccess ||
        (e = dev_malloc((void **)&SB.y, sizeof(double) * N * M2)) != hipSuccess ||
        (e = dev_malloc((void **)&SB.ctoff, sizeof(int32_t) * (ncomp + 1))) != hipSuccess ||
        (e = dev_malloc((void **)&SB.ctids, sizeof(int32_t) * std::max<size_t>(ct_ids.size(), 1))) != hipSuccess ||
        (e = dev_malloc((void **)&SB.acc, N)) != hipSuccess ||
        (e = hipMemcpy(SB.nodes, nd.data(), sizeof(NodeDev) * N, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(SB.y, yv.data(), sizeof(double) * N * M2, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(SB.ctoff, ct_off.data(), sizeof(int32_t) * (ncomp + 1), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (ct_ids.size() &&
         (e = hipMemcpy(SB.ctids, ct_ids.data(), sizeof(int32_t) * ct_ids.size(), hipMemcpyHostToDevice)) !=
             hipSuccess))
      return hip_fail(e, "build step upload");
    {
      dim3 grid((unsigned)std::min<int64_t>((N + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK, 65535)), block(256);
      const int opl = (M2 + WAVE - 1) / WAVE;
#define HIER(OPLV)                                                                                             \
  hipLaunchKernelGGL(k_hierarchize_fp64<OPLV>, grid, block, 0, (hipStream_t)0, D.tups, D.tab, D.alpha, M2, m, \
                     SB.ctoff, SB.ctids, SB.nodes, N, SB.y, P->eps_gamma, SB.acc)
      if (opl <= 1) HIER(1);
      else if (opl <= 2) HIER(2);
      else if (opl <= 4) HIER(4);
      else HIER(8);
#undef HIER
      e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpy(acc.data(), SB.acc, N, hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) return hip_fail(e, "k_hierarchize_fp64");
    SB.free_hier();
    clk.lap(PhaseClock::HIER);
    // ---- register the new rows; append their level multi-indices ----
    std::vector<int32_t> tab_new;
    int64_t t0 = 0;
    while (t0 < N) {
      int64_t t1 = t0;
      while (t1 < N && nn[t1].comp == nn[t0].comp && nn[t1].lvkey == nn[t0].lvkey) ++t1;
      CompState &c = C[nn[t0].comp];
      TupDesc T{};
      T.w = 1.0;
      T.row_base = (int32_t)(rows_used + t0);
      T.comp = nn[t0].comp;
      T.k = (uint8_t)c.k;
      T.lsum = (uint8_t)step;
      int64_t ncells = 1;
      for (int q = 0; q < c.k; ++q) {
        T.dims[q] = (int16_t)c.dims[q];
        T.lv[q] = nn[t0].key.l[q];
        ncells <<= (T.lv[q] - 1);
      }
      const int64_t nr = t1 - t0;
      const int64_t base = tab_used + (int64_t)tab_new.size();
      if (nr == ncells) {
        T.kind = TUP_FULL;
      } else if (ncells <= 4 * nr + 64) {
        T.kind = TUP_DENSE;
        T.aux = (int32_t)base;
        tab_new.resize(tab_new.size() + (size_t)ncells, -1);
        for (int64_t t = t0; t < t1; ++t) tab_new[(size_t)(base - tab_used) + nn[t].slot] = (int32_t)(rows_used + t);
      } else {
        T.kind = TUP_HASH;
        int64_t cap = 4;
        while (cap < 2 * nr) cap <<= 1;
        int64_t b2 = base;
        if (b2 & 1) {
          tab_new.push_back(0);
          ++b2;
        }
        T.aux = (int32_t)b2;
        T.mask = (int32_t)(cap - 1);
        const size_t off = (size_t)(b2 - tab_used);
        tab_new.resize(off + 2 * (size_t)cap, 0);
        for (int64_t q = 0; q < cap; ++q) tab_new[off + 2 * q] = (int32_t)HASH_EMPTY;
        for (int64_t t = t0; t < t1; ++t) {
          uint32_t h = slot_hash(nn[t].slot) & (uint32_t)T.mask;
          while ((uint32_t)tab_new[off + 2 * h] != HASH_EMPTY) h = (h + 1) & (uint32_t)T.mask;
          tab_new[off + 2 * h] = (int32_t)nn[t].slot;
          tab_new[off + 2 * h + 1] = (int32_t)(rows_used + t);
        }
      }
      c.tuples.push_back((int32_t)h_tups.size());
      h_tups.push_back(T);
      for (int64_t t = t0; t < t1; ++t) {
        const int32_t local = (int32_t)c.acc.size();
        if (host_refine) c.index.emplace(nn[t].key, local);
        c.acc.push_back(acc[t]);
        for (int q = 0; q < c.k; ++q) {
          c.lv.push_back(nn[t].key.l[q]);
          c.ix.push_back(nn[t].key.i[q]);
        }
        c.build_row.push_back(rows_used + t);
      }
      t0 = t1;
    }
    if (tab_used + (int64_t)tab_new.size() >= (int64_t)INT32_MAX)
      return fail(HDMR_EUNSUPPORTED, "lookup directory exceeds 2^31 entries");
    if ((rc = grow_device(&D.tab, &D.tab_cap, tab_used + (int64_t)tab_new.size(), tab_used))) return rc;
    if (!tab_new.empty())
      HDMR_HIP(hipMemcpy(D.tab + tab_used, tab_new.data(), sizeof(int32_t) * tab_new.size(), hipMemcpyHostToDevice));
    tab_used += (int64_t)tab_new.size();
    const int64_t tups_before = D.tups ? (int64_t)h_tups.size() : 0;
    (void)tups_before;
    if ((rc = grow_device(&D.tups, &D.tups_cap, (int64_t)h_tups.size(), 0))) return rc;
    HDMR_HIP(hipMemcpy(D.tups, h_tups.data(), sizeof(TupDesc) * h_tups.size(), hipMemcpyHostToDevice));
    rows_used += N;
    clk.lap(PhaseClock::DIRECTORY);
    // ---- children of accepted nodes (Sec. 3.1 exclusion rule) ----
    if (!host_refine) {
      // k_refine: at most 2 |S| candidates per accepted node, each child once
      int64_t cap = 0;
      for (int64_t j = 0; j < N; ++j)
        if (acc[j]) cap += 2 * C[nn[j].comp].k;
      if (cap >= (int64_t)INT32_MAX) return fail(HDMR_EUNSUPPORTED, "more than 2^31-1 candidate children in a step");
      if (cap > 0) {
        if ((e = dev_malloc((void **)&SB.kids, sizeof(ChildDev) * cap)) != hipSuccess ||
            (e = dev_malloc((void **)&SB.nkids, sizeof(uint32_t))) != hipSuccess ||
            (e = hipMemsetAsync(SB.nkids, 0, sizeof(uint32_t), (hipStream_t)0)) != hipSuccess)
          return hip_fail(e, "refinement buffers");
        const int64_t ncand = N * 2 * KMAX;
        hipLaunchKernelGGL(k_refine, dim3((unsigned)std::min<int64_t>((ncand + 255) / 256, 16384)), dim3(256), 0,
                           (hipStream_t)0, SB.nodes, SB.acc, N, P->max_level, P->level_rule, P->refine_rule, SB.kids,
                           SB.nkids);
        uint32_t nk = 0;
        if ((e = hipGetLastError()) != hipSuccess ||
            (e = hipMemcpy(&nk, SB.nkids, sizeof(uint32_t), hipMemcpyDeviceToHost)) != hipSuccess)
          return hip_fail(e, "k_refine");
        if ((int64_t)nk > cap) return fail(HDMR_EDEVICE, "k_refine returned more children than candidates");
        std::vector<ChildDev> kids(nk);
        if (nk && (e = hipMemcpy(kids.data(), SB.kids, sizeof(ChildDev) * nk, hipMemcpyDeviceToHost)) != hipSuccess)
          return hip_fail(e, "k_refine children");
        for (const ChildDev &kd : kids) {
          NodeKey key{};
          for (int q = 0; q < KMAX; ++q) {
            key.l[q] = kd.lv[q];
            key.i[q] = kd.ix[q];
          }
          C[(size_t)kd.comp].pending.push_back(key);
        }
      }
    } else {
      // The nodes are grouped by component (nn is sorted by component) and a
      // component's nodes stay in one thread, so each pending list is built in
      // the same order as by one thread.
      std::vector<int64_t> cstart;
      for (int64_t j = 0; j < N; ++j)
        if (j == 0 || nn[j].comp != nn[j - 1].comp) cstart.push_back(j);
      cstart.push_back(N);
      parallel_ranges((int64_t)cstart.size() - 1, 8, [&](int64_t g0, int64_t g1) {
        for (int64_t j = cstart[(size_t)g0]; j < cstart[(size_t)g1]; ++j) {
          if (!acc[j]) continue;
          CompState &c = C[nn[j].comp];
          const NodeKey &key = nn[j].key;
          int32_t ls = 0;
          for (int q = 0; q < c.k; ++q) ls += key.l[q];
          if (P->level_rule == 1 && ls + 1 > P->max_level + c.k - 1) continue;
          for (int q = 0; q < c.k; ++q) {
            if (P->level_rule == 0 && key.l[q] + 1 > P->max_level) continue;
            for (int side = -1; side <= 1; side += 2) {
              NodeKey ch = key;
              ch.l[q] = (uint8_t)(ch.l[q] + 1);
              ch.i[q] = 2 * ch.i[q] + side;
              int npar = 0, nacc = 0;
              for (int p = 0; p < c.k; ++p) {
                if (ch.l[p] <= 1) continue;
                NodeKey par = ch;
                par.l[p] = (uint8_t)(par.l[p] - 1);
                const uint32_t a = (ch.i[p] - 1) / 2, b = (ch.i[p] + 1) / 2;
                par.i[p] = (a & 1u) ? a : b;
                ++npar;
                auto it = c.index.find(par);
                if (it != c.index.end() && c.acc[it->second]) ++nacc;
              }
              const bool admit = P->refine_rule == 0 ? (nacc == npar) : (nacc > 0);
              if (admit) c.pending.push_back(ch);
            }
          }
        }
      });
      parallel_ranges((int64_t)C.size(), 8, [&](int64_t s0, int64_t s1) {
        for (int64_t s = s0; s < s1; ++s) {
          CompState &c = C[(size_t)s];
          if (c.pending.size() < 2) continue;
          std::sort(c.pending.begin(), c.pending.end(), [&](const NodeKey &a, const NodeKey &b) {
            for (int q = 0; q < c.k; ++q)
              if (a.l[q] != b.l[q]) return a.l[q] < b.l[q];
            for (int q = 0; q < c.k; ++q)
              if (a.i[q] != b.i[q]) return a.i[q] < b.i[q];
            return false;
          });
          c.pending.erase(std::unique(c.pending.begin(), c.pending.end()), c.pending.end());
        }
      });
    }
    clk.lap(PhaseClock::CHILDREN);
  }
  return HDMR_OK;
  };  // run_steps
  std::vector<double> f_anchor((size_t)m);
  if (f(anchor.data(), 1, d, f_anchor.data(), m, user) != 0)
    return fail(HDMR_ECALLBACK, "the user function returned an error");
  auto contains = [](const CompState &u, const int32_t *dims, int k) {
    for (int q = 0; q < k; ++q) {
      bool found = false;
      for (int r = 0; r < u.k; ++r) found |= (u.dims[r] == dims[q]);
      if (!found) return false;
    }
    return true;
  };
  std::vector<int> keep;  // kept components (indices into C), in build order
  std::vector<DdsgCandidate> report;
  std::vector<double> report_rho;
  if (!criteria) {
    C = std::move(all);
    for (auto &c : C) add_root(c);
    int rc = run_steps();
    if (rc) return rc;
    for (int s = 0; s < (int)C.size(); ++s) keep.push_back(s);
  } else {
    // Alg. 2: expansion orders in turn; eq (3.19) rejects candidates into Z,
    // eq (3.18) ends the expansion
    int kmax = 0;
    for (const auto &c : all) kmax = std::max(kmax, c.k);
    std::vector<std::vector<int32_t>> Z;
    std::vector<double> below(f_anchor);  // sum of Q f_v over kept v, |v| < k, and Q f_empty = f(xbar)
    for (int k = 1; k <= kmax; ++k) {
      const size_t first = C.size();
      for (const auto &c : all) {
        if (c.k != k) continue;
        bool pruned = false;
        for (const auto &z : Z) {
          CompState zc;
          zc.k = k;
          for (int q = 0; q < k; ++q) zc.dims[q] = c.dims[q];
          pruned |= contains(zc, z.data(), (int)z.size());
        }
        if (pruned) continue;
        CompState nc;
        nc.k = c.k;
        for (int q = 0; q < KMAX; ++q) nc.dims[q] = c.dims[q];
        add_root(nc);
        C.push_back(std::move(nc));
      }
      if (C.size() == first) break;
      int rc = run_steps();
      if (rc) return rc;
      // quadrature of every candidate's component interpolant (u columns)
      const int64_t ncand = (int64_t)(C.size() - first);
      std::vector<int64_t> qoff(1, 0), qrow;
      std::vector<double> qwt;
      for (size_t s = first; s < C.size(); ++s) {
        const CompState &c = C[s];
        for (size_t r = 0; r < c.acc.size(); ++r) {
          int ls = 0;
          for (int q = 0; q < c.k; ++q) ls += c.lv[r * c.k + q];
          qrow.push_back(c.build_row[r]);
          qwt.push_back(std::ldexp(1.0, -ls));
        }
        qoff.push_back((int64_t)qrow.size());
      }
      std::vector<double> Q((size_t)(ncand * m));
      clk.lap(PhaseClock::QUAD);
      {
        int64_t *d_row = nullptr, *d_off = nullptr;
        double *d_wt = nullptr, *d_q = nullptr;
        hipError_t e = dev_malloc((void **)&d_row, sizeof(int64_t) * std::max<size_t>(qrow.size(), 1));
        if (e == hipSuccess) e = dev_malloc((void **)&d_wt, sizeof(double) * std::max<size_t>(qwt.size(), 1));
        if (e == hipSuccess) e = dev_malloc((void **)&d_off, sizeof(int64_t) * qoff.size());
        if (e == hipSuccess) e = dev_malloc((void **)&d_q, sizeof(double) * Q.size());
        if (e == hipSuccess && !qrow.empty())
          e = hipMemcpy(d_row, qrow.data(), sizeof(int64_t) * qrow.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && !qwt.empty())
          e = hipMemcpy(d_wt, qwt.data(), sizeof(double) * qwt.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_off, qoff.data(), sizeof(int64_t) * qoff.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
          hipLaunchKernelGGL(k_quadrature_rows, dim3((unsigned)ncand), dim3(256), 0, (hipStream_t)0, D.alpha, M2, m, m,
                             d_row, d_wt, d_off, d_q);
          e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpy(Q.data(), d_q, sizeof(double) * Q.size(), hipMemcpyDeviceToHost);
        (void)hipFree(d_row);
        (void)hipFree(d_wt);
        (void)hipFree(d_off);
        (void)hipFree(d_q);
        if (e != hipSuccess) return hip_fail(e, "k_quadrature_rows");
      }
      auto norm2 = [&](const double *v) {
        double s2 = 0.0;
        for (int o = 0; o < m; ++o) s2 += v[o] * v[o];
        return std::sqrt(s2);
      };
      const double denom = norm2(below.data());
      std::vector<double> sum_k((size_t)m, 0.0);
      for (int64_t j = 0; j < ncand; ++j) {
        const CompState &c = C[first + (size_t)j];
        DdsgCandidate rec{};
        rec.k = c.k;
        for (int q = 0; q < KMAX; ++q) rec.dims[q] = q < c.k ? c.dims[q] : -1;
        rec.eta = std::numeric_limits<double>::quiet_NaN();
        bool kept = true;
        if (k >= 2 && P->eps_eta > 0.0) {
          rec.eta = norm2(&Q[(size_t)(j * m)]) / denom;
          kept = rec.eta > P->eps_eta;   // strict, as the text states
        }
        rec.kept = kept ? 1 : 0;
        report.push_back(rec);
        if (kept) {
          keep.push_back((int)(first + (size_t)j));
          for (int o = 0; o < m; ++o) sum_k[(size_t)o] += Q[(size_t)(j * m + o)];
        } else {
          Z.emplace_back(c.dims, c.dims + c.k);
        }
      }
      const double rho = norm2(sum_k.data()) / denom;
      report_rho.push_back(rho);
      for (int o = 0; o < m; ++o) below[(size_t)o] += sum_k[(size_t)o];
      clk.lap(PhaseClock::QUAD);
      if (P->eps_rho > 0.0 && !(rho > P->eps_rho)) break;   // continue only while rho > eps_rho
    }
  }
  // ---- assemble the model from the kept components ----
  const int nkeep = (int)keep.size();
  std::vector<double> weights((size_t)nkeep, 1.0);
  std::vector<double> c0 = f_anchor;
  if (P->form == 1) {
    // eq (4.2): b_i = sum over retained u containing i of (-1)^{|u|-|i|}; the
    // retained family is the kept components plus the empty set.
    int64_t b_empty = 1;
    for (int u : keep) b_empty += (C[u].k % 2) ? -1 : 1;
    for (int s = 0; s < nkeep; ++s) {
      const CompState &cs = C[keep[s]];
      int64_t b = 0;
      for (int u : keep)
        if (contains(C[u], cs.dims, cs.k)) b += ((C[u].k - cs.k) % 2) ? -1 : 1;
      weights[s] = (double)b;
    }
    for (int o = 0; o < m; ++o) c0[o] = (double)b_empty * f_anchor[o];
  }
  std::vector<HostComponent> hc((size_t)nkeep);
  for (int s = 0; s < nkeep; ++s) {
    const CompState &cs = C[keep[s]];
    HostComponent &h = hc[s];
    h.k = cs.k;
    for (int q = 0; q < KMAX; ++q) h.dims[q] = cs.dims[q];
    h.w = weights[s];
    h.n = (int64_t)cs.acc.size();
    h.lv = cs.lv.data();
    h.ix = cs.ix.data();
    h.alpha = nullptr;
    h.src_rows = cs.build_row.data();
  }
  DeviceAlphaSource src{D.alpha, M2, P->form == 0 ? m : 0};
  int rc = make_model(d, m, c0.data(), hc, out, &src);
  if (rc) return rc;
  clk.lap(PhaseClock::ASSEMBLE);
  clk.report(rows_used, f_rows);
  (*out)->ddsg = std::move(report);
  (*out)->ddsg_rho = std::move(report_rho);
  return HDMR_OK;
}

extern "C" int hdmr_build_report(const hdmr_model *model, int32_t *n_candidates, int32_t *n_orders, int32_t *cand_k,
                                 int32_t *cand_dims, double *eta, uint8_t *kept, double *rho) {
  clear_error();
  if (!model || !n_candidates || !n_orders) return fail(HDMR_EINVAL, "hdmr_build_report: null argument");
  *n_candidates = (int32_t)model->ddsg.size();
  *n_orders = (int32_t)model->ddsg_rho.size();
  for (size_t j = 0; j < model->ddsg.size(); ++j) {
    const DdsgCandidate &c = model->ddsg[j];
    if (cand_k) cand_k[j] = c.k;
    if (cand_dims)
      for (int q = 0; q < KMAX; ++q) cand_dims[j * KMAX + q] = c.dims[q];
    if (eta) eta[j] = c.eta;
    if (kept) kept[j] = c.kept;
  }
  if (rho)
    for (size_t j = 0; j < model->ddsg_rho.size(); ++j) rho[j] = model->ddsg_rho[j];
  return HDMR_OK;
}

extern "C" int hdmr_quadrature(const hdmr_model *model, double *q, double *total) {
  clear_error();
  if (!model || (!q && !total)) return fail(HDMR_EINVAL, "hdmr_quadrature: null argument");
  int rc = set_device_of(model);
  if (rc) return rc;
  const int32_t nc = (int32_t)model->comps.size(), m = model->m;
  std::vector<int64_t> off(1, 0), row;
  std::vector<double> wt;
  for (const Component &c : model->comps) {
    for (int64_t r = c.row_begin; r < c.row_end; ++r) {
      int ls = 0;
      for (int k = 0; k < c.k; ++k) ls += model->lv_h[(size_t)(r * KMAX + k)];
      row.push_back(r);
      wt.push_back(std::ldexp(1.0, -ls));
    }
    off.push_back((int64_t)row.size());
  }
  std::vector<double> Q((size_t)std::max(nc, 1) * m, 0.0);
  if (nc > 0) {
    int64_t *d_row = nullptr, *d_off = nullptr;
    double *d_wt = nullptr, *d_q = nullptr;
    hipError_t e = dev_malloc((void **)&d_row, sizeof(int64_t) * std::max<size_t>(row.size(), 1));
    if (e == hipSuccess) e = dev_malloc((void **)&d_wt, sizeof(double) * std::max<size_t>(wt.size(), 1));
    if (e == hipSuccess) e = dev_malloc((void **)&d_off, sizeof(int64_t) * off.size());
    if (e == hipSuccess) e = dev_malloc((void **)&d_q, sizeof(double) * Q.size());
    if (e == hipSuccess && !row.empty())
      e = hipMemcpy(d_row, row.data(), sizeof(int64_t) * row.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !wt.empty()) e = hipMemcpy(d_wt, wt.data(), sizeof(double) * wt.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_quadrature_rows, dim3((unsigned)nc), dim3(256), 0, (hipStream_t)0, model->alpha, model->ms,
                         0, m, d_row, d_wt, d_off, d_q);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(Q.data(), d_q, sizeof(double) * (size_t)nc * m, hipMemcpyDeviceToHost);
    (void)hipFree(d_row);
    (void)hipFree(d_wt);
    (void)hipFree(d_off);
    (void)hipFree(d_q);
    if (e != hipSuccess) return hip_fail(e, "k_quadrature_rows");
  }
  if (q) std::memcpy(q, Q.data(), sizeof(double) * (size_t)nc * m);
  if (total) {
    for (int o = 0; o < m; ++o) {
      double t = model->c0_h[(size_t)o];
      for (int32_t c = 0; c < nc; ++c) t += model->comps[(size_t)c].w * Q[(size_t)c * m + o];
      total[o] = t;
    }
  }
  return HDMR_OK;
}
