// Device helpers shared by the evaluation, mixed-precision and build kernels.
#pragma once

#include "hdmr_internal.h"

namespace hdmr {

constexpr int WAVE = 64;
constexpr int WAVES_PER_BLOCK = 4;

// Active cell of level l at coordinate x: c = min(floor(x 2^l), 2^l - 1)
// (clamped to the domain), odd index i = c | 1, t = x 2^l - i (exact),
// phi = max(0, 1 - |t|) is eq (3.1).  Outside [0,1] phi is 0.
__device__ __forceinline__ void active_cell(double x, int l, uint32_t &half, double &phi, double &t,
                                            uint32_t &c) {
  double scale = (double)(1u << l);
  double xl = x * scale;
  double cf = fmin(fmax(floor(xl), 0.0), scale - 1.0);
  c = (uint32_t)cf;
  t = xl - (double)(c | 1u);
  phi = fmax(0.0, 1.0 - fabs(t));
  half = c >> 1;
}

__device__ __forceinline__ int32_t lookup_row(const TupDesc &T, uint32_t slot, const int32_t *__restrict__ tab) {
  if (T.kind == TUP_FULL) return T.row_base + (int32_t)slot;
  if (T.kind == TUP_DENSE) return tab[T.aux + (int64_t)slot];
  const int2 *ht = reinterpret_cast<const int2 *>(tab + T.aux);
  uint32_t h = slot_hash(slot) & (uint32_t)T.mask;
  for (;;) {
    int2 e = ht[h];
    if ((uint32_t)e.x == slot) return e.y;
    if ((uint32_t)e.x == HASH_EMPTY) return -1;
    h = (h + 1) & (uint32_t)T.mask;
  }
}

// One group of level multi-indices, one per lane (lane < 0: none): the
// basis product at the staged point xs (eq (3.1)-(3.2)) and the row of the
// active cell through the directory (-1 if not stored).
__device__ __forceinline__ void group_lookup(const ModelView &M, const double *xs, int lane, const TupDesc &T,
                                             int32_t &row, double &w) {
  row = -1;
  w = 0.0;
  if (lane < 0 || T.k == 0) return;
  double ww = T.w;
  uint32_t slot = 0;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    if (q < T.k) {
      uint32_t half, c;
      double phi, tt;
      active_cell(xs[T.dims[q]], T.lv[q], half, phi, tt, c);
      ww *= phi;
      slot = (slot << (T.lv[q] - 1)) | half;
    }
  }
  w = ww;
  if (ww != 0.0) row = lookup_row(T, slot, M.tab);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Make LDS writes of one lane visible to the other lanes of the same wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

template <int OW>
__device__ __forceinline__ double reduce_groups(double v) {
#pragma unroll
  for (int off = OW; off < WAVE; off <<= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}


}  // namespace hdmr
