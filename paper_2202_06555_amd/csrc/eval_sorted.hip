// Cell-sorted evaluation (the large-batch path of hdmr_eval, FP64).
//
// Every point of one finest cell of a component's dimensions activates
// exactly the same rows (one odd index per level and dimension, eq (3.3)).
// Per pass (one component of the largest order plus the lower-order
// components inside its dimensions):
//   keys    : the cell of every point in the key dimensions (<= 16 bits);
//   sort    : radix sort of (key, point) pairs, so points of one cell are
//             neighbours in the sorted order;
//   contract: a wavefront takes 64 consecutive sorted points, one per lane.
//             Per level multi-index of the pass (a wave-uniform loop) every
//             lane finds its active cell, its basis weight w = w_S prod phi
//             (eq (3.1), eq (3.2)) and its row through the directory, and
//             accumulates w * alpha[row, :] (eq (3.6)) in FP64 registers.
//             Lanes of one cell read the same directory entries and surplus
//             rows, so these loads are served once per wave from L1.  The
//             sum is added to the point's FP64 output row (the first pass
//             writes c0 + sum).
// Before the passes the points are transposed to dimension-major order (a
// pass reads only its key columns) and NaN points are flagged; after them
// flagged points get NaN outputs.
#include <cstdlib>
#include <cstring>

#include <hipcub/hipcub.hpp>

#include "kernels_common.h"

namespace hdmr {

namespace {

constexpr int RBATCH = 64;           // rows contracted per batch
constexpr int CELLCAP = RBATCH + 64; // discovered rows held in LDS per wave



__global__ void k_transpose(const double *__restrict__ X, int64_t n, int d, double *__restrict__ XT,
                            uint8_t *__restrict__ nanflag) {
  __shared__ double tile[32][33];
  const int64_t p0 = (int64_t)blockIdx.x * 32;
  const int q0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t p = p0 + r;
    const int q = q0 + tx;
    double v = 0.0;
    if (p < n && q < d) {
      v = X[p * d + q];
      if (v != v) nanflag[p] = 1;
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int q = q0 + r;
    const int64_t p = p0 + tx;
    if (p < n && q < d) XT[(int64_t)q * n + p] = tile[tx][r];
  }
}

__global__ void k_fill_u8(uint8_t *__restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = 0;
}
__global__ void k_fill_u32(uint32_t *__restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = 0;
}

__device__ __forceinline__ uint32_t cell_of(double x, int c) {
  const double scale = (double)(1u << c);
  return (uint32_t)fmin(fmax(floor(x * scale), 0.0), scale - 1.0);
}

__global__ void k_keys(const double *__restrict__ XT, int64_t n, Pass P, uint16_t *__restrict__ key,
                       int32_t *__restrict__ idx) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    uint32_t kk = 0;
    for (int q = 0; q < P.k; ++q) kk |= cell_of(XT[(int64_t)P.dims[q] * n + p], P.cell_lv[q]) << P.shift[q];
    key[p] = (uint16_t)kk;
    idx[p] = (int32_t)p;
  }
}

// Coordinates of the pass's key dimensions in sorted order (dimension-major).
__global__ void k_gather_sorted(const double *__restrict__ XT, int64_t n, Pass P, const int32_t *__restrict__ spid,
                                double *__restrict__ sx) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t pid = spid[i];
    for (int q = 0; q < P.k; ++q) sx[(int64_t)q * n + i] = XT[(int64_t)P.dims[q] * n + pid];
  }
}

__global__ void k_nan_fix(double *__restrict__ F, const uint8_t *__restrict__ nanflag, int64_t n, int m) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * m; e += (int64_t)gridDim.x * blockDim.x)
    if (nanflag[e / m]) F[e] = __builtin_nan("");
}

__device__ __forceinline__ double pick(const double (&x)[KMAX], int pos) {
  return pos == 0 ? x[0] : pos == 1 ? x[1] : pos == 2 ? x[2] : x[3];
}

// Cell bounds from the sorted keys: [start, end) of every nonempty cell.
__global__ void k_bounds(const uint16_t *__restrict__ ks, int64_t n, uint32_t *__restrict__ start,
                         uint32_t *__restrict__ end) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint16_t k = ks[i];
    if (i == 0 || ks[i - 1] != k) start[k] = (uint32_t)i;
    if (i == n - 1 || ks[i + 1] != k) end[k] = (uint32_t)(i + 1);
  }
}

__global__ void k_tile_counts(const uint32_t *__restrict__ start, const uint32_t *__restrict__ end, int nbins,
                              uint32_t *__restrict__ ntile) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nbins) ntile[b] = (end[b] - start[b] + WAVE - 1) / WAVE;
}

__global__ void k_write_tiles(const uint32_t *__restrict__ start, const uint32_t *__restrict__ end,
                              const uint32_t *__restrict__ ntile, const uint32_t *__restrict__ toff, int nbins,
                              int4 *__restrict__ tiles, uint32_t *__restrict__ ntiles) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  const uint32_t s0 = start[b], cnt = end[b] - start[b];
  for (uint32_t t = 0; t < ntile[b]; ++t)
    tiles[toff[b] + t] = make_int4(b, (int)(s0 + t * WAVE), (int)min(cnt - t * WAVE, (uint32_t)WAVE), 0);
  if (b == nbins - 1) *ntiles = toff[b] + ntile[b];
}

typedef double v4d __attribute__((ext_vector_type(4)));

// The rows of a cell as found by the discovery step.
struct CellRows {
  double w[CELLCAP];            // w_S
  double sc[CELLCAP][KMAX];     // 2^l per dimension
  double ix[CELLCAP][KMAX];     // i per dimension
  int32_t row[CELLCAP];
  int32_t k[CELLCAP];
  int32_t pos[CELLCAP][KMAX];   // key position of each dimension
};

struct TileLds {
  CellRows rows;
  double xs[WAVE][KMAX];
  int32_t pid[WAVE];
};

// One wavefront per tile (<= 64 sorted points of one cell).
//   discovery: lanes over the pass's level multi-indices find the cell's rows
//     (one candidate cell per level multi-index, more when the cell is coarser
//     than the level), ballot + prefix compaction into LDS;
//   operands : the rows' surpluses for the wave's 16-output column tiles go
//     straight into the MFMA B-operand registers in one burst (each lane
//     holds distinct elements: 4 rows x 16 columns per k-step and tile);
//   contract : per 16-point row tile, each lane forms its A-operand weight
//     w = w_S prod phi (eq (3.1), eq (3.2)) for (point, row) and the wave
//     runs FP64 MFMA 16x16x4 over the cell's rows (eq (3.6));
//   update   : the 16 x 16 output tiles are added to the FP64 output rows
//     (prefetched before the MFMAs; the first pass writes c0 + sum).
template <int NT>
__global__ __launch_bounds__(256, 2) void k_pass_mfma(ModelView M, Pass P, const PassTup *__restrict__ ptups,
                                                   const int4 *__restrict__ tiles, const uint32_t *__restrict__ ntiles_p,
                                                   const int32_t *__restrict__ spid, const double *__restrict__ sx,
                                                   int64_t n, double *__restrict__ F, int first_pass, int o0) {
  constexpr int KS = RBATCH / 4;   // k-steps per batch
  __shared__ TileLds lds[WAVES_PER_BLOCK];
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  TileLds &L = lds[wid];
  const int m = M.m;
  const int kk = lane >> 4, jj = lane & 15;
  const uint32_t ntiles = *ntiles_p;
  const int64_t nw = (int64_t)gridDim.x * WAVES_PER_BLOCK;
  for (int64_t ti = (int64_t)blockIdx.x * WAVES_PER_BLOCK + wid; ti < (int64_t)ntiles; ti += nw) {
    const int4 tile = tiles[ti];
    const uint32_t key = (uint32_t)tile.x;
    const int start = tile.y, count = tile.z;
    {
      const int32_t pid = lane < count ? spid[start + lane] : 0;
      L.pid[lane] = pid;
#pragma unroll
      for (int q = 0; q < KMAX; ++q) L.xs[lane][q] = (lane < count && q < P.k) ? sx[(int64_t)q * n + start + lane] : 0.0;
    }
    uint32_t cellq[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) cellq[q] = q < P.k ? (key >> P.shift[q]) & ((1u << P.cell_lv[q]) - 1u) : 0u;
    bool first = first_pass != 0;
    int rb0 = P.tup_begin;
    uint32_t rcand = 0;
    bool done = rb0 >= P.tup_end;
    int nrows = 0;
    for (;;) {
      // ---- discovery (resumable) until a batch of RBATCH rows is complete ----
      while (!done && nrows < RBATCH) {
        const int j = rb0 + lane;
        TupDesc T{};
        PassTup PT{};
        uint32_t lo[KMAX] = {0, 0, 0, 0}, cnt[KMAX] = {1, 1, 1, 1}, ncand = 0;
        if (j < P.tup_end) {
          PT = ptups[j];
          T = M.tups[PT.tup];
          ncand = 1;
#pragma unroll
          for (int q = 0; q < KMAX; ++q) {
            if (q < T.k) {
              const int c = P.cell_lv[PT.pos[q]], l = T.lv[q];
              const uint32_t cell = cellq[PT.pos[q]];
              if (l <= c) {
                lo[q] = (cell >> (c - l)) >> 1;
                cnt[q] = 1;
              } else {
                lo[q] = (cell << (l - c)) >> 1;
                cnt[q] = 1u << (l - c - 1);
              }
              ncand *= cnt[q];
            }
          }
        }
        uint32_t maxc = ncand;
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) maxc = max(maxc, (uint32_t)__shfl_xor((int)maxc, off, WAVE));
        uint32_t cand = rcand;
        for (; cand < maxc && nrows < RBATCH; ++cand) {
          int32_t row = -1;
          uint32_t half[KMAX] = {0, 0, 0, 0};
          if (cand < ncand) {
            uint32_t rem = cand, slot = 0;
#pragma unroll
            for (int q = KMAX - 1; q >= 0; --q)
              if (q < T.k) {
                half[q] = lo[q] + rem % cnt[q];
                rem /= cnt[q];
              }
#pragma unroll
            for (int q = 0; q < KMAX; ++q)
              if (q < T.k) slot = (slot << (T.lv[q] - 1)) | half[q];
            row = lookup_row(T, slot, M.tab);
          }
          const bool hit = row >= 0;
          const uint64_t mask = ballot(hit);
          if (hit) {
            const int e = nrows + lanes_below(mask);
            L.rows.w[e] = T.w;
            L.rows.row[e] = row;
            L.rows.k[e] = T.k;
#pragma unroll
            for (int q = 0; q < KMAX; ++q) {
              L.rows.pos[e][q] = PT.pos[q];
              L.rows.sc[e][q] = (double)(1u << (T.lv[q] ? T.lv[q] : 1));
              L.rows.ix[e][q] = (double)(2u * half[q] + 1u);
            }
          }
          nrows += __popcll(mask);
        }
        if (cand < maxc) {
          rcand = cand;
        } else {
          rcand = 0;
          rb0 += WAVE;
          done = rb0 >= P.tup_end;
        }
      }
      wave_sync();
      const int R = min(nrows, RBATCH);
      if (R > 0 || (done && first)) {
        const int Rp = (R + 3) & ~3;
        // B operands of the whole batch, one burst
        double b[KS][NT];
#pragma unroll
        for (int s4 = 0; s4 < KS; ++s4) {
          const int r = s4 * 4 + kk;
          const int32_t row = r < R ? L.rows.row[r] : -1;
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int o = o0 + nt * 16 + jj;
            b[s4][nt] = (row >= 0 && o < m) ? M.alpha[(int64_t)row * M.ms + o] : 0.0;
          }
        }
        const int nmt = (count + 15) >> 4;
        for (int mt = 0; mt < nmt; ++mt) {
          v4d acc[NT];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[nt] = v4d{0.0, 0.0, 0.0, 0.0};
          const int pa = mt * 16 + jj;   // this lane's A-operand point
#pragma unroll
          for (int s4 = 0; s4 < KS; ++s4) {
            if (s4 * 4 < Rp) {
              const int r = s4 * 4 + kk;
              double w = 0.0;
              if (r < R && pa < count) {
                w = L.rows.w[r];
                const int k = L.rows.k[r];
#pragma unroll
                for (int q = 0; q < KMAX; ++q)
                  if (q < k) w *= fmax(0.0, 1.0 - fabs(L.xs[pa][L.rows.pos[r][q]] * L.rows.sc[r][q] - L.rows.ix[r][q]));
              }
#pragma unroll
              for (int nt = 0; nt < NT; ++nt) acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(w, b[s4][nt], acc[nt], 0, 0, 0);
            }
          }
          // the first contraction of a point writes c0 + sum; later ones add
          // with device atomics (no value returned, so the wave never waits;
          // one tile owns a point within a pass, passes run in order)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int pt = mt * 16 + kk + 4 * i;
            if (pt < count) {
              double *fr = F + (int64_t)L.pid[pt] * m;
#pragma unroll
              for (int nt = 0; nt < NT; ++nt) {
                const int o = o0 + nt * 16 + jj;
                if (o < m) {
                  if (first)
                    fr[o] = M.c0[o] + acc[nt][i];
                  else
                    atomicAdd(fr + o, acc[nt][i]);
                }
              }
            }
          }
        }
        first = false;
      }
      // rows past the batch move to the front
      const int rest = nrows - R;
      if (rest > 0) {
        double tw = 0.0, tsc[KMAX], tix[KMAX];
        int32_t trow = 0, tk = 0, tpos[KMAX];
        if (lane < rest) {
          const int e = R + lane;
          tw = L.rows.w[e];
          trow = L.rows.row[e];
          tk = L.rows.k[e];
#pragma unroll
          for (int q = 0; q < KMAX; ++q) {
            tsc[q] = L.rows.sc[e][q];
            tix[q] = L.rows.ix[e][q];
            tpos[q] = L.rows.pos[e][q];
          }
        }
        wave_sync();
        if (lane < rest) {
          L.rows.w[lane] = tw;
          L.rows.row[lane] = trow;
          L.rows.k[lane] = tk;
#pragma unroll
          for (int q = 0; q < KMAX; ++q) {
            L.rows.sc[lane][q] = tsc[q];
            L.rows.ix[lane][q] = tix[q];
            L.rows.pos[lane][q] = tpos[q];
          }
        }
      }
      wave_sync();
      nrows = rest;
      if (done && nrows == 0) break;
    }
  }
}

template <typename T>
int ws_alloc(T **p, size_t count, hipStream_t s) {
  HDMR_HIP(hipMallocAsync((void **)p, std::max<size_t>(count, 1) * sizeof(T), s));
  return HDMR_OK;
}

}  // namespace

int eval_sorted_fp64(const hdmr_model *model, const double *X, int64_t n, double *F, hipStream_t stream) {
  const ModelView M = model->view();
  const int d = M.d, m = M.m;
  if (n >= (int64_t)INT32_MAX) return fail(HDMR_EUNSUPPORTED, "n >= 2^31 points in one call");
  double *xt = nullptr;
  uint8_t *nanflag = nullptr;
  double *sxv = nullptr;
  uint16_t *key = nullptr, *key_s = nullptr;
  int32_t *idx = nullptr, *spid = nullptr;
  uint32_t *bstart = nullptr, *bend = nullptr, *ntile = nullptr, *toff = nullptr, *ntiles = nullptr;
  int4 *tiles = nullptr;
  void *tmp = nullptr;
  size_t tmp_sort = 0, tmp_scan = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_sort, key, key_s, idx, spid, (int)n, 0, 16, stream) !=
          hipSuccess ||
      hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_scan, ntile, toff, 65536, stream) != hipSuccess)
    return fail(HDMR_EDEVICE, "hipcub temporary storage query failed");
  const size_t max_tiles = (size_t)(n / WAVE) + 65536 + 1;
  const size_t tmp_bytes = std::max(tmp_sort, tmp_scan);
  int rc = HDMR_OK;
  auto release = [&]() {
    void *ptrs[] = {xt, sxv, nanflag, key, key_s, idx, spid, bstart, bend, ntile, toff, ntiles, tiles, tmp};
    for (void *p : ptrs) (void)hipFreeAsync(p, stream);
  };
  if ((rc = ws_alloc(&xt, (size_t)n * d, stream)) || (rc = ws_alloc(&nanflag, (size_t)n, stream)) ||
      (rc = ws_alloc(&sxv, (size_t)n * KMAX, stream)) ||
      (rc = ws_alloc(&key, (size_t)n, stream)) || (rc = ws_alloc(&key_s, (size_t)n, stream)) ||
      (rc = ws_alloc(&idx, (size_t)n, stream)) || (rc = ws_alloc(&spid, (size_t)n, stream)) ||
      (rc = ws_alloc(&bstart, (size_t)65536, stream)) || (rc = ws_alloc(&bend, (size_t)65536, stream)) ||
      (rc = ws_alloc(&ntile, (size_t)65536, stream)) || (rc = ws_alloc(&toff, (size_t)65536, stream)) ||
      (rc = ws_alloc(&ntiles, (size_t)1, stream)) || (rc = ws_alloc(&tiles, max_tiles, stream)) ||
      (rc = ws_alloc((char **)&tmp, tmp_bytes, stream))) {
    release();
    return rc;
  }
  const unsigned gs = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fill_u8, dim3(gs), dim3(256), 0, stream, nanflag, n);
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((n + 31) / 32), (unsigned)((d + 31) / 32)), dim3(256), 0, stream,
                     X, n, d, xt, nanflag);
  int first = 1;
  hipError_t e = hipSuccess;
  for (const Pass &P : model->passes) {
    const int nbins = 1 << P.key_bits;
    hipLaunchKernelGGL(k_keys, dim3(gs), dim3(256), 0, stream, xt, n, P, key, idx);
    size_t tb = tmp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(tmp, tb, key, key_s, idx, spid, (int)n, 0, P.key_bits, stream);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_fill_u32, dim3((nbins + 255) / 256), dim3(256), 0, stream, bstart, (int64_t)nbins);
    hipLaunchKernelGGL(k_fill_u32, dim3((nbins + 255) / 256), dim3(256), 0, stream, bend, (int64_t)nbins);
    hipLaunchKernelGGL(k_bounds, dim3(gs), dim3(256), 0, stream, key_s, n, bstart, bend);
    hipLaunchKernelGGL(k_tile_counts, dim3((nbins + 255) / 256), dim3(256), 0, stream, bstart, bend, nbins, ntile);
    tb = tmp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(tmp, tb, ntile, toff, nbins, stream);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_write_tiles, dim3((nbins + 255) / 256), dim3(256), 0, stream, bstart, bend, ntile, toff,
                       nbins, tiles, ntiles);
    hipLaunchKernelGGL(k_gather_sorted, dim3(gs), dim3(256), 0, stream, xt, n, P, spid, sxv);
    for (int o0 = 0; o0 < m; o0 += 32) {
      const int nt = (std::min(32, m - o0) + 15) / 16;
#define PASS(NTV)                                                                                                   \
  hipLaunchKernelGGL(k_pass_mfma<NTV>, dim3(4096), dim3(256), 0, stream, M, P, model->pass_tups, tiles, ntiles, spid, \
                     sxv, n, F, first, o0)
      if (nt == 1) PASS(1);
      else PASS(2);
#undef PASS
    }
    first = 0;
  }
  if (e == hipSuccess && first) e = hipErrorInvalidValue;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_nan_fix, dim3(gs), dim3(256), 0, stream, F, nanflag, n, m);
    e = hipGetLastError();
  }
  release();
  if (e != hipSuccess) return hip_fail(e, "sorted evaluation");
  return HDMR_OK;
}

}  // namespace hdmr
