// BF16 MLP surrogate: training and inference kernels (BF16 MFMA GEMMs with
// fused epilogues, GELU, MSE gradient, Adam) and the per-output routing
// between the network and the sparse-grid interpolant.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "../../include/hdmr_surrogate.h"
#include "hdmr_internal.h"

using namespace hdmr;

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NL = 4;          // linear layers
constexpr int TM = 64, TN = 64, TK = 32;
constexpr int LK = TK + 8;     // LDS row stride (bf16): 80-byte rows keep 16-byte alignment
constexpr int CHUNK_ROWS = 65536;  // rows per inference chunk
constexpr int DW_SPLIT_MAX = 16;    // K slices of the weight-gradient GEMM
constexpr int DW_BLOCKS = 512;      // workgroups the split aims for
constexpr int COLSUM_CHUNKS = 64;   // row chunks of the bias-gradient reduction
constexpr int WIDE128_MIN_TILES = 1024;  // workgroups of the 128 x 128 tile kernel (four per CU)

inline int64_t pad8(int64_t x) { return (x + 7) & ~(int64_t)7; }

// GELU(z) = 0.5 z (1 + erf(z / sqrt 2)) = 0.5 (z + |z| erf(|z| / sqrt 2)),
// with erf on [0, inf) by Abramowitz & Stegun 7.1.26 (|error| <= 1.5e-7,
// far below one BF16 ulp of the stored activation): branch-free, one
// hardware reciprocal and one hardware exp2.
__device__ __forceinline__ float gelu_f(float z) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
  const float poly =
      t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
  const float erf_abs = fmaf(-poly, __builtin_amdgcn_exp2f(-x * x * 1.4426950408889634f), 1.0f);
  return 0.5f * fmaf(fabsf(z), erf_abs, z);
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

enum Epi : int { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_DH = 2, EPI_DW = 3 };

// C (M x N) = A (M x K) * B (K x N), BF16 operands, FP32 accumulation.
// A: TA = 0 -> A[m * lda + k]; TA = 1 -> A[k * lda + m].
// B: TB = 0 -> B[k * ldb + n]; TB = 1 -> B[n * ldb + k].
// lda and ldb are multiples of 8 (16-byte aligned rows).
struct Gemm {
  const bf16 *A;
  int64_t lda;
  const bf16 *B;
  int64_t ldb;
  int M, N, K;
  const float *bias;  // HIDDEN, OUT
  float *Z;           // HIDDEN: pre-activations out (may be NULL); DH: pre-activations in
  int64_t ldz;
  bf16 *H;            // HIDDEN: GELU(z) out; DH: dz out
  int64_t ldh;
  float *C;           // OUT, DW (DW: slice z writes C + z * M * ldc)
  int64_t ldc;
  int kslice;         // K per workgroup slice along blockIdx.z (a multiple of TK)
};

// Stage a 64 x 32 tile of a [rows][k] operand into LDS (row-major, k
// contiguous).  KC = 1: the matrix stores k contiguously (rows x k);
// KC = 0: it stores rows contiguously (k x rows).
template <int KC>
__device__ __forceinline__ void stage(bf16 (*dst)[LK], const bf16 *__restrict__ src, int64_t ld, int r0, int k0,
                                      int R, int K, int t) {
  if (KC) {
    const int r = t >> 2, kv = (t & 3) * 8;
    const int gr = r0 + r, gk = k0 + kv;
    bf16x8 v;
    if (gr < R && gk + 8 <= K) {
      v = *reinterpret_cast<const bf16x8 *>(src + (int64_t)gr * ld + gk);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (gr < R && gk + e < K) ? src[(int64_t)gr * ld + gk + e] : (bf16)0.0f;
    }
    *reinterpret_cast<bf16x8 *>(&dst[r][kv]) = v;
  } else {
    const int k = t >> 3, rv = (t & 7) * 8;
    const int gk = k0 + k, gr = r0 + rv;
    bf16x8 v;
    if (gk < K && gr + 8 <= R) {
      v = *reinterpret_cast<const bf16x8 *>(src + (int64_t)gk * ld + gr);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (gk < K && gr + e < R) ? src[(int64_t)gk * ld + gr + e] : (bf16)0.0f;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) dst[rv + e][k] = v[e];
  }
}

// Bias of the NB column tiles a lane stores (HIDDEN, OUT), loaded up front.
template <int EPI, int NB>
__device__ __forceinline__ void load_bias(const Gemm &g, int c0, int i, float (&bv)[NB]) {
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int col = c0 + 16 * b + i;
    bv[b] = ((EPI == EPI_HIDDEN || EPI == EPI_OUT) && col < g.N) ? g.bias[col] : 0.f;
  }
}

// Fused epilogue of a wave's NA x NB MFMA tiles (rows r0 + 16 a + 4 kg + r,
// columns c0 + 16 b + i).  Every operand is read before the first store, so
// the loads overlap instead of each waiting behind a store it might alias.
template <int EPI, int NA, int NB>
__device__ __forceinline__ void store_tiles(const Gemm &g, const f32x4 (&acc)[NA][NB], int r0, int c0, int i, int kg,
                                            const float (&bv)[NB]) {
  float zv[NA][NB][4];
  if constexpr (EPI == EPI_DH) {
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + 16 * a + 4 * kg + r, col = c0 + 16 * b + i;
          zv[a][b][r] = (row < g.M && col < g.N) ? g.Z[(int64_t)row * g.ldz + col] : 0.f;
        }
  }
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 16 * a + 4 * kg + r, col = c0 + 16 * b + i;
        if (row >= g.M || col >= g.N) continue;
        const float v = acc[a][b][r];
        if constexpr (EPI == EPI_HIDDEN) {
          const float z = v + bv[b];
          if (g.Z) g.Z[(int64_t)row * g.ldz + col] = z;
          g.H[(int64_t)row * g.ldh + col] = (bf16)gelu_f(z);
        } else if constexpr (EPI == EPI_OUT) {
          g.C[(int64_t)row * g.ldc + col] = v + bv[b];
        } else if constexpr (EPI == EPI_DH) {
          g.H[(int64_t)row * g.ldh + col] = (bf16)(v * gelu_grad_f(zv[a][b][r]));
        } else {
          g.C[((int64_t)blockIdx.z * g.M + row) * g.ldc + col] = v;  // slice blockIdx.z of a split-K product
        }
      }
}

// 64 x 64 output tile per workgroup of 4 waves; each wave a 32 x 32 quarter
// (2 x 2 MFMA 16x16x32 tiles).
template <int TA, int TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
  __shared__ __attribute__((aligned(16))) bf16 sA[TM][LK];
  __shared__ __attribute__((aligned(16))) bf16 sB[TN][LK];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int i = lane & 15, kg = lane >> 4;
  float bv[2];
  load_bias<EPI, 2>(g, n0 + wn, i, bv);
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kb = blockIdx.z * g.kslice, ke = min(g.K, kb + g.kslice);
  for (int k0 = kb; k0 < ke; k0 += TK) {
    __syncthreads();
    stage<TA == 0>(sA, g.A, g.lda, m0, k0, g.M, g.K, t);
    stage<TB == 1>(sB, g.B, g.ldb, n0, k0, g.N, g.K, t);
    __syncthreads();
    bf16x8 av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = *reinterpret_cast<const bf16x8 *>(&sA[wm + 16 * a + i][8 * kg]);
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = *reinterpret_cast<const bf16x8 *>(&sB[wn + 16 * b + i][8 * kg]);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
  // lane holds rows 4 kg + r, column i of each 16 x 16 tile
  store_tiles<EPI, 2, 2>(g, acc, m0 + wm, n0 + wn, i, kg, bv);
}

// Large-tile kernel for tall products: a (2 WT) x (2 WT) output tile per
// workgroup of 4 waves, each wave a WT x WT quarter of (WT/16)^2 MFMA tiles,
// k in steps of 64 through two LDS buffers; the next step is fetched into
// registers while the current one is multiplied (one barrier per step).
// Launched with WT = 64 (two workgroups per CU); WT = 128 (one workgroup,
// accumulators in AGPRs) measured slower on the network's products.
constexpr int BK = 64, LB = BK;  // 128-byte LDS rows, swizzled
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// LDS position of column col of an operand row: the 16-byte piece q of row
// r sits at piece q ^ ((r >> 1) & 7), so the 16 rows one MFMA operand read
// touches (and the two rows a 16-lane store touches) hit distinct banks.
__device__ __forceinline__ int lds_col(int row, int col) { return (((col >> 3) ^ ((row >> 1) & 7)) << 3) | (col & 7); }

// ROWS / 32 16-byte pieces per thread of a ROWS x 64 operand tile; KC as in
// stage().  Rows at or past R and k at or past kend read as zero.  Row
// strides are multiples of 8 elements that cover the stored width, so
// fetch_tile() reads every piece from a clamped address inside its row;
// piece_valid() counts the piece's valid elements and put_tile() masks off
// the rest once the load has landed.
template <int KC, int ROWS>
__device__ __forceinline__ int piece_valid(int c, int r0, int k0, int R, int kend) {
  constexpr int PK = ROWS / 8;  // pieces per k when rows are contiguous
  if (KC) {
    const int gr = r0 + (c >> 3), gk = k0 + (c & 7) * 8;
    return gr < R ? kend - gk : 0;
  }
  const int gk = k0 + c / PK, gr = r0 + (c % PK) * 8;
  return gk < kend ? R - gr : 0;
}

template <int KC, int ROWS>
__device__ __forceinline__ void fetch_tile(u32x4 (&r)[ROWS / 32], const bf16 *__restrict__ src, int64_t ld, int r0,
                                           int k0, int R, int kend, int t) {
  constexpr int PK = ROWS / 8;
#pragma unroll
  for (int j = 0; j < ROWS / 32; ++j) {
    const int c = t + 256 * j;
    int64_t off;
    if (KC) {
      const int gr = r0 + (c >> 3), gk = k0 + (c & 7) * 8;
      off = (int64_t)min(gr, R - 1) * ld + min((int64_t)gk, ld - 8);
    } else {
      const int gk = k0 + c / PK, gr = r0 + (c % PK) * 8;
      off = (int64_t)min(gk, kend - 1) * ld + min((int64_t)gr, ld - 8);
    }
    r[j] = *reinterpret_cast<const u32x4 *>(src + off);
  }
}

// Masks off the elements past the bounds (piece_valid(), the same geometry
// as the fetch) and writes the pieces to LDS.
template <int KC, int ROWS>
__device__ __forceinline__ void put_tile(bf16 (*dst)[LB], const u32x4 (&r)[ROWS / 32], int r0, int k0, int R, int kend,
                                         int t) {
  constexpr int PK = ROWS / 8;
#pragma unroll
  for (int j = 0; j < ROWS / 32; ++j) {
    const int c = t + 256 * j;
    const int nv = piece_valid<KC, ROWS>(c, r0, k0, R, kend);
    u32x4 v = r[j];
    if (nv < 8) {
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] &= (2 * q < nv ? 0xFFFFu : 0u) | (2 * q + 1 < nv ? 0xFFFF0000u : 0u);
    }
    if (KC) {
      const int row = c >> 3;
      *reinterpret_cast<u32x4 *>(&dst[row][lds_col(row, (c & 7) * 8)]) = v;
    } else {
      const bf16x8 e8 = __builtin_bit_cast(bf16x8, v);
      const int rv = (c % PK) * 8, k = c / PK;
#pragma unroll
      for (int e = 0; e < 8; ++e) dst[rv + e][lds_col(rv + e, k)] = e8[e];
    }
  }
}

// One 64-deep k step of a wave's WT x WT quarter from LDS.
template <int WT>
__device__ __forceinline__ void mma_tile(const bf16 (*sa)[LB], const bf16 (*sb)[LB], f32x4 (&acc)[WT / 16][WT / 16],
                                         int wm, int wn, int i, int kg) {
  constexpr int NT = WT / 16;
#pragma unroll
  for (int ks = 0; ks < BK; ks += 32) {
    bf16x8 av[NT];
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const int row = wm + 16 * a + i;
      av[a] = *reinterpret_cast<const bf16x8 *>(&sa[row][lds_col(row, ks + 8 * kg)]);
    }
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      const int row = wn + 16 * b + i;
      const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&sb[row][lds_col(row, ks + 8 * kg)]);
#pragma unroll
      for (int a = 0; a < NT; ++a) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv, acc[a][b], 0, 0, 0);
    }
  }
}

template <int WT>
constexpr size_t tile_lds_bytes() {
  // operands (two buffers of 2 WT rows each for A and B) or half the output
  // tile (WT rows of 2 WT FP32 values plus a 16-byte pad)
  return std::max<size_t>(2 * 4 * WT * LB * sizeof(bf16), (size_t)WT * (2 * WT + 4) * sizeof(float));
}

template <int TA, int TB, int EPI, int WT>
__global__ __launch_bounds__(256, WT == 64 ? 2 : 1) void k_gemm_wide(Gemm g) {
  constexpr int NT = WT / 16, BT = 2 * WT;
  __shared__ __attribute__((aligned(16))) unsigned char lds[tile_lds_bytes<WT>()];
  bf16 (*sA)[BT][LB] = reinterpret_cast<bf16 (*)[BT][LB]>(lds);
  bf16 (*sB)[BT][LB] = reinterpret_cast<bf16 (*)[BT][LB]>(lds + 2 * BT * LB * sizeof(bf16));
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // consecutive workgroups land on different XCDs (each with its own L2):
  // give every XCD a contiguous run of tiles so the tiles sharing a row
  // block of A share that L2
  const int gx = (int)gridDim.x, T = gx * (int)gridDim.y;
  int L = (int)blockIdx.x + gx * (int)blockIdx.y;
  if ((T & 7) == 0) L = (L & 7) * (T >> 3) + (L >> 3);
  const int m0 = (L / gx) * BT, n0 = (L % gx) * BT;
  const int wm = (w >> 1) * WT, wn = (w & 1) * WT;
  const int i = lane & 15, kg = lane >> 4;
  const int kb = blockIdx.z * g.kslice, ke = min(g.K, kb + g.kslice);
  float bv[NT];
  load_bias<EPI, NT>(g, n0 + wn, i, bv);
  f32x4 acc[NT][NT];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (kb < ke) {
    u32x4 ra[BT / 32], rb[BT / 32];
    fetch_tile<TA == 0, BT>(ra, g.A, g.lda, m0, kb, g.M, ke, t);
    fetch_tile<TB == 1, BT>(rb, g.B, g.ldb, n0, kb, g.N, ke, t);
    put_tile<TA == 0, BT>(sA[0], ra, m0, kb, g.M, ke, t);
    put_tile<TB == 1, BT>(sB[0], rb, n0, kb, g.N, ke, t);
    __syncthreads();
    int cur = 0;
    for (int k0 = kb; k0 < ke; k0 += BK) {
      const bool more = k0 + BK < ke;
      if (more) {
        fetch_tile<TA == 0, BT>(ra, g.A, g.lda, m0, k0 + BK, g.M, ke, t);
        fetch_tile<TB == 1, BT>(rb, g.B, g.ldb, n0, k0 + BK, g.N, ke, t);
      }
      mma_tile<WT>(sA[cur], sB[cur], acc, wm, wn, i, kg);
      if (more) {
        put_tile<TA == 0, BT>(sA[cur ^ 1], ra, m0, k0 + BK, g.M, ke, t);
        put_tile<TB == 1, BT>(sB[cur ^ 1], rb, n0, k0 + BK, g.N, ke, t);
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  if constexpr (EPI == EPI_HIDDEN || EPI == EPI_OUT) {
    // Stage the FP32 products plus bias in LDS, one half of the tile (the
    // rows of two waves) at a time, then sweep whole rows: each thread takes
    // 4 consecutive values, applies the activation and writes them as one
    // piece.  Lane-scattered 2- or 4-byte stores would split every cache
    // line of the output between several store instructions.  Columns past
    // N hold zeros (masked operands, zero bias) and are written to H and C
    // only up to their padded row strides.
    constexpr int TS = BT + 4;      // LDS row stride (floats) of the staged half
    constexpr int PPR = BT / 4;     // 4-value pieces per row
    static_assert((size_t)WT * TS * sizeof(float) <= sizeof(lds), "output half exceeds LDS");
    float *tile = reinterpret_cast<float *>(lds);
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
      __syncthreads();
      if ((w >> 1) == half) {
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
          for (int b = 0; b < NT; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) tile[(16 * a + 4 * kg + r) * TS + wn + 16 * b + i] = acc[a][b][r] + bv[b];
      }
      __syncthreads();
#pragma unroll 4
      for (int q = 0; q < WT * PPR / 256; ++q) {
        const int c = t + 256 * q;
        const int lr = c / PPR, lc = (c % PPR) * 4;
        const int row = m0 + half * WT + lr, col = n0 + lc;
        if (row >= g.M) continue;
        const f32x4 z = *reinterpret_cast<const f32x4 *>(&tile[lr * TS + lc]);
        if constexpr (EPI == EPI_HIDDEN) {
          if (g.Z) {
            float *zp = g.Z + (int64_t)row * g.ldz + col;
            if (col + 4 <= g.N && (g.ldz & 3) == 0) {
              *reinterpret_cast<f32x4 *>(zp) = z;
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (col + e < g.N) zp[e] = z[e];
            }
          }
          if (col < g.ldh) {
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            bf16x4 h;
#pragma unroll
            for (int e = 0; e < 4; ++e) h[e] = (bf16)gelu_f(z[e]);
            *reinterpret_cast<bf16x4 *>(g.H + (int64_t)row * g.ldh + col) = h;
          }
        } else {
          if (col < g.ldc) *reinterpret_cast<f32x4 *>(g.C + (int64_t)row * g.ldc + col) = z;
        }
      }
    }
  } else {
    store_tiles<EPI, NT, NT>(g, acc, m0 + wm, n0 + wn, i, kg, bv);
  }
}

// Rows idx[r] (or row0 + r when idx is NULL) of X (n x d, FP64) -> H (rows
// x ldh, BF16).  One wave per row, lanes across its columns.
__global__ void k_rows_to_bf16(const double *__restrict__ X, int d, const int64_t *__restrict__ idx, int64_t row0,
                               int64_t rows, bf16 *__restrict__ H, int64_t ldh) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); r < rows;
       r += (int64_t)gridDim.x * (blockDim.x >> 6)) {
    const int64_t src = idx ? idx[r] : row0 + r;
    const double *x = X + src * d;
    bf16 *h = H + r * ldh;
    for (int q = lane; q < d; q += 64) h[q] = (bf16)(float)x[q];
  }
}

// Standardised targets of the batch rows: T[r][o] = (Y[idx[r]][o] - mean[o]) / std[o].
__global__ void k_targets(const double *__restrict__ Y, int m, const int64_t *__restrict__ idx, int64_t rows,
                          const float *__restrict__ mean, const float *__restrict__ stdv, float *__restrict__ T) {
  const int64_t total = rows * m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / m;
    const int o = (int)(e - r * m);
    T[e] = (float)((Y[idx[r] * m + o] - (double)mean[o]) / (double)stdv[o]);
  }
}

// G = 2 (out - T) / (rows m) (BF16), and the batch loss sum((out - T)^2) / (rows m) added to *loss.
__global__ void k_loss_grad(const float *__restrict__ out, int64_t ldo, const float *__restrict__ T, int m,
                            int64_t rows, bf16 *__restrict__ G, int64_t ldg, float *__restrict__ loss) {
  __shared__ float part[256];
  const float inv = 1.0f / (float)(rows * m);
  float s = 0.f;
  const int64_t total = rows * m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / m;
    const int o = (int)(e - r * m);
    const float diff = out[r * ldo + o] - T[e];
    G[r * ldg + o] = (bf16)(2.0f * diff * inv);
    s += diff * diff;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, part[0] * inv);
}

// Bias gradient db[c] = sum_r G[r][c] in two deterministic stages.  Stage 1:
// workgroup (x, y) sums columns 64x .. 64x+63 over row chunk y, 4 waves on
// interleaved rows, into part[y][c].
__global__ __launch_bounds__(256) void k_colsum_part(const bf16 *__restrict__ G, int64_t ldg, int64_t rows, int N,
                                                     float *__restrict__ part) {
  __shared__ float red[4][64];
  const int cl = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  const int64_t per = (rows + gridDim.y - 1) / gridDim.y;
  const int64_t r0 = (int64_t)blockIdx.y * per, r1 = min(rows, r0 + per);
  float s = 0.f;
  if (c < N)
    for (int64_t r = r0 + wv; r < r1; r += 4) s += (float)G[r * ldg + c];
  red[wv][cl] = s;
  __syncthreads();
  if (wv == 0 && c < N) part[(int64_t)blockIdx.y * N + c] = (red[0][cl] + red[1][cl]) + (red[2][cl] + red[3][cl]);
}

// Stage 2 (also the split-K reduction of the weight gradient): out[e] = sum_z part[z * len + e].
__global__ void k_sum_slices(const float *__restrict__ part, int slices, int64_t len, float *__restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < slices; ++z) s += part[(int64_t)z * len + e];
    out[e] = s;
  }
}

__global__ void k_fill_f32(float *__restrict__ a, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = v;
}

// Adam on the packed FP32 parameters (t counted from 1).
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ mom,
                       float *__restrict__ vel, int64_t n, float lr, float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * mom[i] + (1.f - b1) * gi;
    const float vi = b2 * vel[i] + (1.f - b2) * gi * gi;
    mom[i] = mi;
    vel[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// BF16 copy of a row-major (rows x cols) FP32 matrix with row stride ld.
__global__ void k_to_bf16(const float *__restrict__ W, int rows, int cols, bf16 *__restrict__ Wb, int64_t ld) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols;
    Wb[r * ld + (e - r * cols)] = (bf16)W[e];
  }
}

// Y[row0 + r][o] = out[r][o] * std[o] + mean[o] (FP64).
// Y[r][o] = out[r][o] std[o] + mean[o] (FP64); one wave per row.
__global__ void k_destd(const float *__restrict__ out, int64_t ldo, int64_t rows, int m, const float *__restrict__ mean,
                        const float *__restrict__ stdv, double *__restrict__ Y) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); r < rows;
       r += (int64_t)gridDim.x * (blockDim.x >> 6)) {
    const float *o_ = out + r * ldo;
    double *y = Y + r * m;
    for (int o = lane; o < m; o += 64) y[o] = (double)o_[o] * (double)stdv[o] + (double)mean[o];
  }
}

// Per-output mean and standard deviation of Y (n x m), one block per output.
__global__ void k_moments(const double *__restrict__ Y, int64_t n, int m, float *__restrict__ mean,
                          float *__restrict__ stdv) {
  __shared__ double s1[256], s2[256];
  const int o = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    const double v = Y[r * m + o];
    a += v;
    b += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s1[threadIdx.x] += s1[threadIdx.x + off];
      s2[threadIdx.x] += s2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mu = s1[0] / (double)n;
    const double var = std::max(s2[0] / (double)n - mu * mu, 0.0);
    mean[o] = (float)mu;
    stdv[o] = (float)std::max(std::sqrt(var), 1e-12);
  }
}

// Y[r][cols[j]] = A[r][j] (+ P[r][cols[j]] when P is given), r < n, j < k.
__global__ void k_scatter_cols(const double *__restrict__ A, int k, const int32_t *__restrict__ cols,
                               const double *__restrict__ P, int64_t n, int m, double *__restrict__ Y) {
  const int64_t total = n * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / k;
    const int c = cols[e - r * k];
    Y[r * m + c] = A[e] + (P ? P[r * m + c] : 0.0);
  }
}

// max over rows of |A[r][o] + P[r][o] - T[r][o]| per output (one block per output).
__global__ void k_maxerr(const double *__restrict__ A, const double *__restrict__ P, const double *__restrict__ T,
                         int64_t n, int m, double *__restrict__ err) {
  __shared__ double s[256];
  const int o = blockIdx.x;
  double mx = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    const double e = fabs(A[r * m + o] + P[r * m + o] - T[r * m + o]);
    mx = e > mx || e != e ? e : mx;
  }
  s[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const double a = s[threadIdx.x], b = s[threadIdx.x + off];
      s[threadIdx.x] = (b > a || b != b) ? b : a;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) err[o] = s[0];
}

// Per-point gate: rows whose two network predictions P, P2 differ by more
// than tau in any of the k served columns are listed in idx (order of
// discovery; count in *cnt, which must start at 0).
__global__ void k_gate_rows(const double *__restrict__ P, const double *__restrict__ P2, int64_t n, int m,
                            const int32_t *__restrict__ cols, int k, double tau, int64_t *__restrict__ idx,
                            unsigned long long *__restrict__ cnt) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    bool out = false;
    for (int j = 0; j < k; ++j) {
      const int c = cols[j];
      const double dlt = fabs(P[r * m + c] - P2[r * m + c]);
      out |= !(dlt <= tau);
    }
    if (out) idx[atomicAdd(cnt, 1ull)] = r;
  }
}

__global__ void k_zero_count(unsigned long long *c) {
  if (threadIdx.x == 0) *c = 0ull;
}

// Xg[i] = X[idx[i]] (rows of d values).
__global__ void k_gather_rows(const double *__restrict__ X, const int64_t *__restrict__ idx, int64_t ng, int d,
                              double *__restrict__ Xg) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ng * d; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / d;
    Xg[e] = X[idx[i] * d + (e - i * d)];
  }
}

// Y[idx[i]][cols[j]] = A[i][j].
__global__ void k_scatter_rows(const double *__restrict__ A, const int64_t *__restrict__ idx, int64_t ng, int k,
                               const int32_t *__restrict__ cols, int m, double *__restrict__ Y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ng * k; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / k;
    Y[idx[i] * m + cols[e - i * k]] = A[e];
  }
}

unsigned grid_of(int64_t total) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 16384)); }
// workgroups for one-wave-per-row kernels (4 rows per workgroup of 256)
// K slices of the out x in weight gradient: enough 64 x 64 tiles for
// DW_BLOCKS workgroups, at most DW_SPLIT_MAX slices.
int64_t dw_split(int64_t out, int64_t in) {
  const int64_t tiles = ((out + TM - 1) / TM) * ((in + TN - 1) / TN);
  return std::min<int64_t>(DW_SPLIT_MAX, std::max<int64_t>(1, (DW_BLOCKS + tiles - 1) / tiles));
}

unsigned row_grid(int64_t rows) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((rows + 3) / 4, 16384)); }

template <int TA, int TB, int EPI>
hipError_t gemm(const Gemm &g, hipStream_t s) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  Gemm gg = g;
  unsigned slices = 1;
  if (EPI == EPI_DW && gg.kslice > 0)
    slices = (unsigned)((gg.K + gg.kslice - 1) / gg.kslice);
  else
    gg.kslice = std::max(gg.K, 1);
  if constexpr (EPI != EPI_DW) {
    // 128 x 128 tiles once they give every CU four workgroups, else 64 x 64
    const int64_t t128 = (int64_t)((g.N + 127) / 128) * ((g.M + 127) / 128);
    if (t128 >= WIDE128_MIN_TILES) {
      const dim3 grid((unsigned)((g.N + 127) / 128), (unsigned)((g.M + 127) / 128), 1);
      hipLaunchKernelGGL((k_gemm_wide<TA, TB, EPI, 64>), grid, dim3(256), 0, s, gg);
      return hipGetLastError();
    }
  }
  const dim3 grid((unsigned)((g.N + TN - 1) / TN), (unsigned)((g.M + TM - 1) / TM), slices);
  hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, gg);
  return hipGetLastError();
}

}  // namespace

struct mlp_model {
  int device = 0;
  int32_t d = 0, w = 0, m = 0;
  int32_t in[NL] = {0, 0, 0, 0}, out[NL] = {0, 0, 0, 0};
  int64_t ldin[NL] = {0, 0, 0, 0};  // padded input widths (BF16 row strides)
  int64_t woff[NL] = {0, 0, 0, 0}, boff[NL] = {0, 0, 0, 0};
  int64_t nparam = 0;
  float *p = nullptr, *g = nullptr, *mom = nullptr, *vel = nullptr;  // packed FP32
  bf16 *wb[NL] = {nullptr, nullptr, nullptr, nullptr};              // BF16 weight copies (out x ldin)
  float *mean = nullptr, *stdv = nullptr;
  bool have_std = false;
  int64_t adam_t = 0;
  // batch workspace
  int64_t cap = 0;
  bf16 *h[NL] = {nullptr, nullptr, nullptr, nullptr};  // layer inputs (cap x ldin[l])
  float *z[NL - 1] = {nullptr, nullptr, nullptr};      // hidden pre-activations (cap x w)
  float *outv = nullptr;                               // cap x pad8(m)
  float *tgt = nullptr;                                // cap x m
  bf16 *gb[2] = {nullptr, nullptr};                    // output / pre-activation gradients (cap x pad8(max(w, m)))
  float *loss = nullptr;                               // 1 float per step slot
  int64_t loss_cap = 0;
  float *ws = nullptr;                                 // split-K slices / bias-gradient partials
  int64_t ws_len = 0;

  ~mlp_model() {
    void *ptrs[] = {p, g, mom, vel, mean, stdv, wb[0], wb[1], wb[2], wb[3], outv, tgt, gb[0], gb[1], loss,
                    h[0], h[1], h[2], h[3], z[0], z[1], z[2], ws};
    for (void *q : ptrs) (void)hipFree(q);
  }

  int reserve(int64_t rows) {
    if (rows <= cap) return HDMR_OK;
    for (auto &q : h) { (void)hipFree(q); q = nullptr; }
    for (auto &q : z) { (void)hipFree(q); q = nullptr; }
    for (auto &q : gb) { (void)hipFree(q); q = nullptr; }
    (void)hipFree(outv);
    (void)hipFree(tgt);
    outv = tgt = nullptr;
    cap = 0;
    const int64_t gw = pad8(std::max(w, m));
    for (int l = 0; l < NL; ++l) HDMR_HIP(dev_malloc((void **)&h[l], sizeof(bf16) * rows * ldin[l]));
    for (int l = 0; l < NL - 1; ++l) HDMR_HIP(dev_malloc((void **)&z[l], sizeof(float) * rows * w));
    for (int q = 0; q < 2; ++q) HDMR_HIP(dev_malloc((void **)&gb[q], sizeof(bf16) * rows * gw));
    HDMR_HIP(dev_malloc((void **)&outv, sizeof(float) * rows * pad8(m)));
    HDMR_HIP(dev_malloc((void **)&tgt, sizeof(float) * rows * m));
    cap = rows;
    return HDMR_OK;
  }

  hipError_t refresh_bf16(hipStream_t s) {
    for (int l = 0; l < NL; ++l)
      hipLaunchKernelGGL(k_to_bf16, dim3(grid_of((int64_t)out[l] * in[l])), dim3(256), 0, s, p + woff[l], out[l],
                         in[l], wb[l], ldin[l]);
    return hipGetLastError();
  }

  // Forward of `rows` staged inputs in h[0]; keeps pre-activations when train.
  hipError_t forward(int64_t rows, bool train, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int l = 0; l < NL && e == hipSuccess; ++l) {
      Gemm gg{};
      gg.A = h[l];
      gg.lda = ldin[l];
      gg.B = wb[l];
      gg.ldb = ldin[l];
      gg.M = (int)rows;
      gg.N = out[l];
      gg.K = in[l];
      gg.bias = p + boff[l];
      if (l < NL - 1) {
        gg.Z = train ? z[l] : nullptr;
        gg.ldz = w;
        gg.H = h[l + 1];
        gg.ldh = ldin[l + 1];
        e = gemm<0, 1, EPI_HIDDEN>(gg, s);
      } else {
        gg.C = outv;
        gg.ldc = pad8(m);
        e = gemm<0, 1, EPI_OUT>(gg, s);
      }
    }
    return e;
  }

  // Backward of the batch (gradient of the output in gb[0]) into g.
  hipError_t backward(int64_t rows, hipStream_t s) {
    hipError_t e = hipSuccess;
    const int64_t gw = pad8(std::max(w, m));
    int cur = 0;
    for (int l = NL - 1; l >= 0 && e == hipSuccess; --l) {
      // dW_l = G^T H_l  (out x in), reduction over the batch
      Gemm dw{};
      dw.A = gb[cur];
      dw.lda = gw;
      dw.B = h[l];
      dw.ldb = ldin[l];
      dw.M = out[l];
      dw.N = in[l];
      dw.K = (int)rows;
      // split K so that the (out x in) tile grid fills the chip; slices go to ws
      const int64_t want = dw_split(out[l], in[l]);
      dw.kslice = (int)(((rows + want - 1) / want + TK - 1) / TK * TK);
      const int slices = (int)((rows + dw.kslice - 1) / dw.kslice);
      const int64_t len = (int64_t)out[l] * in[l];
      dw.C = slices > 1 ? ws : g + woff[l];
      dw.ldc = in[l];
      e = gemm<1, 0, EPI_DW>(dw, s);
      if (e != hipSuccess) break;
      if (slices > 1)
        hipLaunchKernelGGL(k_sum_slices, dim3(grid_of(len)), dim3(256), 0, s, ws, slices, len, g + woff[l]);
      const int chunks = (int)std::min<int64_t>(COLSUM_CHUNKS, std::max<int64_t>(1, rows / 64));
      hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)((out[l] + 63) / 64), (unsigned)chunks), dim3(256), 0, s,
                         gb[cur], gw, rows, out[l], ws);
      hipLaunchKernelGGL(k_sum_slices, dim3(grid_of(out[l])), dim3(256), 0, s, ws, chunks, (int64_t)out[l],
                         g + boff[l]);
      if (l > 0) {
        // dZ_{l-1} = (G W_l) * gelu'(Z_{l-1})
        Gemm dh{};
        dh.A = gb[cur];
        dh.lda = gw;
        dh.B = wb[l];
        dh.ldb = ldin[l];
        dh.M = (int)rows;
        dh.N = in[l];
        dh.K = out[l];
        dh.Z = z[l - 1];
        dh.ldz = w;
        dh.H = gb[cur ^ 1];
        dh.ldh = gw;
        e = gemm<0, 0, EPI_DH>(dh, s);
        cur ^= 1;
      }
    }
    if (e == hipSuccess) e = hipGetLastError();
    return e;
  }

  // Loss gradient of a staged batch (inputs in h[0], targets in tgt) into g;
  // the batch loss is added to *lossp.
  hipError_t grads(int64_t rows, float *lossp, hipStream_t s) {
    hipError_t e = forward(rows, true, s);
    if (e != hipSuccess) return e;
    // few workgroups: each adds its partial loss to one FP32 word
    hipLaunchKernelGGL(k_loss_grad, dim3(std::min(grid_of(rows * m), 512u)), dim3(256), 0, s, outv, pad8(m), tgt, m, rows, gb[0],
                       pad8(std::max(w, m)), lossp);
    return backward(rows, s);
  }
};

struct mlp_route {
  mlp_model *net = nullptr;
  int32_t m = 0, d = 0;
  std::vector<double> err;
  std::vector<int32_t> use;
  std::vector<int32_t> mlp_cols, fb_cols;
  int32_t *d_mlp_cols = nullptr, *d_fb_cols = nullptr;
  hdmr_model *order1 = nullptr;    // order-1 part restricted to the network's outputs
  hdmr_model *fallback = nullptr;  // all components restricted to the other outputs
  // per-point gate: a second network; a point whose two predictions differ by
  // more than gate_tau in any network-served output takes those outputs from
  // served_full (all components, the network's outputs)
  mlp_model *second = nullptr;
  double gate_tau = 0.0;
  hdmr_model *served_full = nullptr;
  int64_t *d_gate_count = nullptr;
  int64_t last_gated = 0;
  ~mlp_route() {
    (void)hipFree(d_mlp_cols);
    (void)hipFree(d_fb_cols);
    (void)hipFree(d_gate_count);
    if (order1) hdmr_free(order1);
    if (fallback) hdmr_free(fallback);
    if (served_full) hdmr_free(served_full);
  }
};

namespace {

int check_dims(int32_t d, int32_t w, int32_t m) {
  if (d < 1 || d > 4096 || m < 1 || m > 4096 || w < 16 || w > 4096)
    return fail(HDMR_EINVAL, "mlp: d, m must be in [1, 4096] and width in [16, 4096]");
  return HDMR_OK;
}

int64_t count_params(int32_t d, int32_t w, int32_t m) {
  return (int64_t)w * d + w + 2 * ((int64_t)w * w + w) + (int64_t)m * w + m;
}

int set_device(const mlp_model *net) {
  int cur = -1;
  HDMR_HIP(hipGetDevice(&cur));
  if (cur != net->device) HDMR_HIP(hipSetDevice(net->device));
  return HDMR_OK;
}

int check_ptr(const void *p) {
  if (((uintptr_t)p & 7) != 0) return fail(HDMR_EINVAL, "misaligned pointer");
  return HDMR_OK;
}

// Network prediction (de-standardised FP64) of rows [0, n) of X into Y, in chunks.
int forward_rows(const mlp_model *cnet, const double *X, int64_t n, double *Y, hipStream_t s) {
  mlp_model *net = const_cast<mlp_model *>(cnet);  // workspace only
  int rc = net->reserve(std::min<int64_t>(std::max<int64_t>(n, 1), CHUNK_ROWS));
  if (rc) return rc;
  for (int64_t r0 = 0; r0 < n; r0 += net->cap) {
    const int64_t rows = std::min<int64_t>(net->cap, n - r0);
    hipLaunchKernelGGL(k_rows_to_bf16, dim3(row_grid(rows)), dim3(256), 0, s, X, net->d,
                       (const int64_t *)nullptr, r0, rows, net->h[0], net->ldin[0]);
    hipError_t e = net->forward(rows, false, s);
    if (e != hipSuccess) return hip_fail(e, "mlp forward");
    hipLaunchKernelGGL(k_destd, dim3(row_grid(rows)), dim3(256), 0, s, net->outv, pad8(net->m), rows,
                       net->m, net->mean, net->stdv, Y + r0 * net->m);
  }
  HDMR_HIP(hipGetLastError());
  return HDMR_OK;
}

}  // namespace

extern "C" {

int mlp_param_count(int32_t d, int32_t width, int32_t m, int64_t *count) {
  clear_error();
  if (!count) return fail(HDMR_EINVAL, "null count");
  int rc = check_dims(d, width, m);
  if (rc) return rc;
  *count = count_params(d, width, m);
  return HDMR_OK;
}

int mlp_create(int32_t d, int32_t width, int32_t m, const float *params, mlp_model **out) {
  clear_error();
  if (!params || !out) return fail(HDMR_EINVAL, "mlp_create: null argument");
  *out = nullptr;
  int rc = check_dims(d, width, m);
  if (rc) return rc;
  mlp_model *net = new mlp_model();
  net->d = d;
  net->w = width;
  net->m = m;
  const int32_t dims[NL + 1] = {d, width, width, width, m};
  int64_t o = 0;
  for (int l = 0; l < NL; ++l) {
    net->in[l] = dims[l];
    net->out[l] = dims[l + 1];
    net->ldin[l] = pad8(dims[l]);
    net->woff[l] = o;
    o += (int64_t)dims[l + 1] * dims[l];
    net->boff[l] = o;
    o += dims[l + 1];
  }
  net->nparam = o;
  hipError_t e = hipGetDevice(&net->device);
  if (e == hipSuccess) e = dev_malloc((void **)&net->p, sizeof(float) * o);
  if (e == hipSuccess) e = dev_malloc((void **)&net->g, sizeof(float) * o);
  if (e == hipSuccess) e = dev_malloc((void **)&net->mom, sizeof(float) * o);
  if (e == hipSuccess) e = dev_malloc((void **)&net->vel, sizeof(float) * o);
  if (e == hipSuccess) e = dev_malloc((void **)&net->mean, sizeof(float) * m);
  if (e == hipSuccess) e = dev_malloc((void **)&net->stdv, sizeof(float) * m);
  if (e == hipSuccess) e = dev_malloc((void **)&net->loss, sizeof(float) * 1);
  net->loss_cap = 1;
  for (int l = 0; l < NL && e == hipSuccess; ++l)
    e = dev_malloc((void **)&net->wb[l], sizeof(bf16) * net->out[l] * net->ldin[l]);
  // only layers whose weight gradient is split need slices (wide layers fill
  // the chip unsplit)
  int64_t wsl = (int64_t)COLSUM_CHUNKS * std::max(width, m);
  for (int l = 0; l < NL; ++l) {
    const int64_t want = dw_split(net->out[l], net->in[l]);
    if (want > 1) wsl = std::max<int64_t>(wsl, want * net->out[l] * net->in[l]);
  }
  if (e == hipSuccess) e = dev_malloc((void **)&net->ws, sizeof(float) * wsl);
  net->ws_len = wsl;
  if (e == hipSuccess) e = hipMemcpy(net->p, params, sizeof(float) * o, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(o)), dim3(256), 0, (hipStream_t)0, net->mom, o, 0.f);
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(o)), dim3(256), 0, (hipStream_t)0, net->vel, o, 0.f);
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(m)), dim3(256), 0, (hipStream_t)0, net->mean, (int64_t)m, 0.f);
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(m)), dim3(256), 0, (hipStream_t)0, net->stdv, (int64_t)m, 1.f);
    // BF16 weight copies: zero the padding columns once, then convert
    for (int l = 0; l < NL && e == hipSuccess; ++l)
      e = hipMemset(net->wb[l], 0, sizeof(bf16) * net->out[l] * net->ldin[l]);
    if (e == hipSuccess) e = net->refresh_bf16((hipStream_t)0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  if (e != hipSuccess) {
    delete net;
    return hip_fail(e, "mlp_create");
  }
  *out = net;
  return HDMR_OK;
}

int mlp_get_params(const mlp_model *net, float *params) {
  clear_error();
  if (!net || !params) return fail(HDMR_EINVAL, "mlp_get_params: null argument");
  int rc = set_device(net);
  if (rc) return rc;
  HDMR_HIP(hipDeviceSynchronize());
  HDMR_HIP(hipMemcpy(params, net->p, sizeof(float) * net->nparam, hipMemcpyDeviceToHost));
  return HDMR_OK;
}

int mlp_set_standardization(mlp_model *net, const float *mean, const float *stdev) {
  clear_error();
  if (!net || !mean || !stdev) return fail(HDMR_EINVAL, "mlp_set_standardization: null argument");
  for (int o = 0; o < net->m; ++o)
    if (!(stdev[o] > 0.f) || !std::isfinite(mean[o])) return fail(HDMR_EINVAL, "standard deviations must be > 0");
  int rc = set_device(net);
  if (rc) return rc;
  HDMR_HIP(hipMemcpy(net->mean, mean, sizeof(float) * net->m, hipMemcpyHostToDevice));
  HDMR_HIP(hipMemcpy(net->stdv, stdev, sizeof(float) * net->m, hipMemcpyHostToDevice));
  net->have_std = true;
  return HDMR_OK;
}

int mlp_fit_standardization(mlp_model *net, const double *Y, int64_t n, hdmr_stream_t stream) {
  clear_error();
  if (!net || !Y || n < 2) return fail(HDMR_EINVAL, "mlp_fit_standardization: needs >= 2 targets");
  if (check_ptr(Y)) return HDMR_EINVAL;
  int rc = set_device(net);
  if (rc) return rc;
  hipLaunchKernelGGL(k_moments, dim3((unsigned)net->m), dim3(256), 0, (hipStream_t)stream, Y, n, net->m, net->mean,
                     net->stdv);
  HDMR_HIP(hipGetLastError());
  net->have_std = true;
  return HDMR_OK;
}

int mlp_get_standardization(const mlp_model *net, float *mean, float *stdev) {
  clear_error();
  if (!net || !mean || !stdev) return fail(HDMR_EINVAL, "mlp_get_standardization: null argument");
  int rc = set_device(net);
  if (rc) return rc;
  HDMR_HIP(hipDeviceSynchronize());
  HDMR_HIP(hipMemcpy(mean, net->mean, sizeof(float) * net->m, hipMemcpyDeviceToHost));
  HDMR_HIP(hipMemcpy(stdev, net->stdv, sizeof(float) * net->m, hipMemcpyDeviceToHost));
  return HDMR_OK;
}

int mlp_forward(const mlp_model *net, const double *X, int64_t n, double *Y, hdmr_stream_t stream) {
  clear_error();
  if (!net || n < 0 || (n > 0 && (!X || !Y))) return fail(HDMR_EINVAL, "mlp_forward: bad argument");
  if (check_ptr(X) || check_ptr(Y)) return HDMR_EINVAL;
  if (n == 0) return HDMR_OK;
  int rc = set_device(net);
  if (rc) return rc;
  return forward_rows(net, X, n, Y, (hipStream_t)stream);
}

int mlp_loss_grads(mlp_model *net, const double *X, const double *Y, const int64_t *idx, int32_t batch,
                   float *grads, float *loss, hdmr_stream_t stream) {
  clear_error();
  if (!net || !X || !Y || !idx || batch < 1 || !grads || !loss) return fail(HDMR_EINVAL, "mlp_loss_grads: bad argument");
  int rc = set_device(net);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (!net->have_std) return fail(HDMR_EINVAL, "mlp_loss_grads: standardisation not set");
  if ((rc = net->reserve(batch))) return rc;
  hipLaunchKernelGGL(k_rows_to_bf16, dim3(row_grid(batch)), dim3(256), 0, s, X, net->d, idx,
                     (int64_t)0, (int64_t)batch, net->h[0], net->ldin[0]);
  hipLaunchKernelGGL(k_targets, dim3(grid_of((int64_t)batch * net->m)), dim3(256), 0, s, Y, net->m, idx,
                     (int64_t)batch, net->mean, net->stdv, net->tgt);
  hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(256), 0, s, net->loss, (int64_t)1, 0.f);
  hipError_t e = net->grads(batch, net->loss, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(grads, net->g, sizeof(float) * net->nparam, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(loss, net->loss, sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "mlp_loss_grads");
  return HDMR_OK;
}

int mlp_train(mlp_model *net, const double *X, const double *Y, const int64_t *order, int64_t steps, int32_t batch,
              float lr0, float *losses, hdmr_stream_t stream) {
  clear_error();
  if (!net || !X || !Y || !order || steps < 0 || batch < 1 || !(lr0 > 0.f))
    return fail(HDMR_EINVAL, "mlp_train: bad argument");
  if (check_ptr(X) || check_ptr(Y) || check_ptr(order)) return HDMR_EINVAL;
  if (steps == 0) return HDMR_OK;
  int rc = set_device(net);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (!net->have_std) return fail(HDMR_EINVAL, "mlp_train: set the standardisation first (mlp_set_standardization)");
  if ((rc = net->reserve(batch))) return rc;
  if (losses && net->loss_cap < steps) {
    (void)hipFree(net->loss);
    net->loss = nullptr;
    net->loss_cap = 0;
    HDMR_HIP(dev_malloc((void **)&net->loss, sizeof(float) * steps));
    net->loss_cap = steps;
  }
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_of(net->loss_cap)), dim3(256), 0, s, net->loss, net->loss_cap, 0.f);
  hipError_t e = hipSuccess;
  for (int64_t st = 0; st < steps && e == hipSuccess; ++st) {
    const int64_t *idx = order + st * batch;
    hipLaunchKernelGGL(k_rows_to_bf16, dim3(row_grid(batch)), dim3(256), 0, s, X, net->d, idx,
                       (int64_t)0, (int64_t)batch, net->h[0], net->ldin[0]);
    hipLaunchKernelGGL(k_targets, dim3(grid_of((int64_t)batch * net->m)), dim3(256), 0, s, Y, net->m, idx,
                       (int64_t)batch, net->mean, net->stdv, net->tgt);
    e = net->grads(batch, net->loss + (losses ? st : 0), s);
    if (e != hipSuccess) break;
    const int64_t t = ++net->adam_t;
    const float lr = (float)(0.5 * lr0 * (1.0 + std::cos(M_PI * (double)st / (double)steps)));
    const float c1 = (float)(1.0 - std::pow(0.9, (double)t)), c2 = (float)(1.0 - std::pow(0.999, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(grid_of(net->nparam)), dim3(256), 0, s, net->p, net->g, net->mom, net->vel,
                       net->nparam, lr, c1, c2);
    e = net->refresh_bf16(s);
  }
  if (e == hipSuccess && losses) {
    e = hipMemcpyAsync(losses, net->loss, sizeof(float) * steps, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e != hipSuccess) return hip_fail(e, "mlp_train");
  return HDMR_OK;
}

void mlp_free(mlp_model *net) {
  if (!net) return;
  (void)set_device(net);
  (void)hipDeviceSynchronize();
  delete net;
}

int hdmr_model_select(const hdmr_model *src, int32_t n_comps, const int32_t *comps, int32_t n_outs,
                      const int32_t *outs, int32_t with_c0, hdmr_model **out) {
  clear_error();
  if (!src || !out || (comps && n_comps < 0) || (outs && n_outs < 1))
    return fail(HDMR_EINVAL, "hdmr_model_select: bad argument");
  *out = nullptr;
  const int32_t nc_all = (int32_t)src->comps.size(), m = src->m;
  std::vector<int32_t> cs, os;
  if (comps) {
    cs.assign(comps, comps + n_comps);
    for (int32_t c : cs)
      if (c < 0 || c >= nc_all) return fail(HDMR_EINVAL, "hdmr_model_select: component id out of range");
  } else {
    for (int32_t c = 0; c < nc_all; ++c) cs.push_back(c);
  }
  if (outs) {
    os.assign(outs, outs + n_outs);
    for (int32_t o : os)
      if (o < 0 || o >= m) return fail(HDMR_EINVAL, "hdmr_model_select: output id out of range");
  } else {
    for (int32_t o = 0; o < m; ++o) os.push_back(o);
  }
  const int32_t mo = (int32_t)os.size();
  std::vector<double> c0(mo);
  for (int32_t j = 0; j < mo; ++j) c0[j] = with_c0 ? src->c0_h[os[j]] : 0.0;
  std::vector<int32_t> offs(1, 0), dims;
  std::vector<int64_t> npts;
  std::vector<uint8_t> lv;
  std::vector<uint32_t> ix;
  std::vector<double> al, w, tmp;
  for (int32_t c : cs) {
    int64_t n = 0;
    int32_t k = 0, dd[KMAX] = {0, 0, 0, 0};
    double wt = 0.0;
    int rc = hdmr_export_component(src, c, &n, &k, dd, nullptr, nullptr, nullptr, &wt);
    if (rc) return rc;
    const size_t l0 = lv.size(), a0 = al.size();
    lv.resize(l0 + (size_t)(n * k));
    ix.resize(l0 + (size_t)(n * k));
    tmp.resize((size_t)(n * m));
    rc = hdmr_export_component(src, c, &n, &k, dd, lv.data() + l0, ix.data() + l0, tmp.data(), &wt);
    if (rc) return rc;
    al.resize(a0 + (size_t)(n * mo));
    for (int64_t r = 0; r < n; ++r)
      for (int32_t j = 0; j < mo; ++j) al[a0 + (size_t)(r * mo + j)] = tmp[(size_t)(r * m + os[j])];
    dims.insert(dims.end(), dd, dd + k);
    offs.push_back(offs.back() + k);
    npts.push_back(n);
    w.push_back(wt);
  }
  return hdmr_model_from_surpluses(src->d, mo, c0.data(), (int32_t)cs.size(), offs.data(), dims.data(), npts.data(),
                                   lv.data(), ix.data(), al.data(), w.data(), out);
}

int mlp_route_create(mlp_model *net, const hdmr_model *full, const double *Xval, int64_t nval, double threshold,
                     mlp_route **out) {
  clear_error();
  if (!net || !full || !Xval || nval < 1 || !out || !(threshold >= 0.0))
    return fail(HDMR_EINVAL, "mlp_route_create: bad argument");
  if (full->m != net->m || full->d != net->d) return fail(HDMR_EINVAL, "mlp_route_create: d or m differ");
  *out = nullptr;
  int rc = set_device(net);
  if (rc) return rc;
  const int32_t m = net->m;
  // order-1 part of the interpolant (all outputs)
  std::vector<int32_t> c1;
  for (int32_t c = 0; c < (int32_t)full->comps.size(); ++c)
    if (full->comps[c].k == 1) c1.push_back(c);
  hdmr_model *o1all = nullptr;
  if ((rc = hdmr_model_select(full, (int32_t)c1.size(), c1.data(), 0, nullptr, 1, &o1all))) return rc;
  double *F = nullptr, *A = nullptr, *P = nullptr, *E = nullptr;
  const size_t bytes = sizeof(double) * (size_t)nval * m;
  hipError_t e = dev_malloc((void **)&F, bytes);
  if (e == hipSuccess) e = dev_malloc((void **)&A, bytes);
  if (e == hipSuccess) e = dev_malloc((void **)&P, bytes);
  if (e == hipSuccess) e = dev_malloc((void **)&E, sizeof(double) * m);
  mlp_route *R = nullptr;
  if (e != hipSuccess) {
    rc = hip_fail(e, "mlp_route_create");
  } else if (!(rc = hdmr_eval(full, Xval, nval, F, m, HDMR_PLAIN_FP64, nullptr)) &&
             !(rc = hdmr_eval(o1all, Xval, nval, A, m, HDMR_PLAIN_FP64, nullptr)) &&
             !(rc = forward_rows(net, Xval, nval, P, (hipStream_t)0))) {
    hipLaunchKernelGGL(k_maxerr, dim3((unsigned)m), dim3(256), 0, (hipStream_t)0, A, P, F, nval, m, E);
    R = new mlp_route();
    R->net = net;
    R->m = m;
    R->d = net->d;
    R->err.assign(m, 0.0);
    R->use.assign(m, 0);
    e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(R->err.data(), E, sizeof(double) * m, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = hip_fail(e, "mlp_route_create");
  }
  (void)hipFree(F);
  (void)hipFree(A);
  (void)hipFree(P);
  (void)hipFree(E);
  hdmr_free(o1all);
  if (rc) {
    delete R;
    return rc;
  }
  for (int32_t o = 0; o < m; ++o) {
    R->use[o] = R->err[o] <= threshold ? 1 : 0;
    (R->use[o] ? R->mlp_cols : R->fb_cols).push_back(o);
  }
  if (!R->mlp_cols.empty())
    rc = hdmr_model_select(full, (int32_t)c1.size(), c1.data(), (int32_t)R->mlp_cols.size(), R->mlp_cols.data(), 1,
                           &R->order1);
  if (!rc && !R->fb_cols.empty())
    rc = hdmr_model_select(full, 0, nullptr, (int32_t)R->fb_cols.size(), R->fb_cols.data(), 1, &R->fallback);
  if (!rc) {
    e = dev_malloc((void **)&R->d_mlp_cols, sizeof(int32_t) * std::max<size_t>(1, R->mlp_cols.size()));
    if (e == hipSuccess) e = dev_malloc((void **)&R->d_fb_cols, sizeof(int32_t) * std::max<size_t>(1, R->fb_cols.size()));
    if (e == hipSuccess && !R->mlp_cols.empty())
      e = hipMemcpy(R->d_mlp_cols, R->mlp_cols.data(), sizeof(int32_t) * R->mlp_cols.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !R->fb_cols.empty())
      e = hipMemcpy(R->d_fb_cols, R->fb_cols.data(), sizeof(int32_t) * R->fb_cols.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = hip_fail(e, "mlp_route_create");
  }
  if (rc) {
    delete R;
    return rc;
  }
  *out = R;
  return HDMR_OK;
}

int mlp_route_info(const mlp_route *route, int32_t *n_mlp, double *err, int32_t *use_mlp) {
  clear_error();
  if (!route) return fail(HDMR_EINVAL, "mlp_route_info: null route");
  if (n_mlp) *n_mlp = (int32_t)route->mlp_cols.size();
  if (err) std::memcpy(err, route->err.data(), sizeof(double) * route->m);
  if (use_mlp) std::memcpy(use_mlp, route->use.data(), sizeof(int32_t) * route->m);
  return HDMR_OK;
}

// The per-point gate of a routed evaluation: the second network's
// predictions at X, the rows where the two disagree by more than gate_tau in
// a served output, and the interpolant's values of the served outputs there
// (synchronous: the number of gated rows sizes the evaluation).
static int gate_points(const mlp_route *route, const double *X, int64_t n, const double *P, double *Y,
                       int32_t precision, hipStream_t s) {
  const int32_t m = route->m, k1 = (int32_t)route->mlp_cols.size(), d = route->d;
  double *P2 = nullptr, *Xg = nullptr, *Ag = nullptr;
  int64_t *idx = nullptr;
  unsigned long long ng = 0;
  int rc = HDMR_OK;
  hipError_t e = dev_malloc_async((void **)&P2, sizeof(double) * (size_t)n * m, s);
  if (e == hipSuccess) e = dev_malloc_async((void **)&idx, sizeof(int64_t) * (size_t)n, s);
  if (e != hipSuccess) rc = hip_fail(e, "mlp gate");
  if (!rc) hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, s, (unsigned long long *)route->d_gate_count);
  if (!rc && !(rc = forward_rows(route->second, X, n, P2, s))) {
    hipLaunchKernelGGL(k_gate_rows, dim3(grid_of(n)), dim3(256), 0, s, P, P2, n, m, route->d_mlp_cols, k1,
                       route->gate_tau, idx, (unsigned long long *)route->d_gate_count);
    e = hipMemcpyAsync(&ng, route->d_gate_count, sizeof(ng), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e, "mlp gate");
  }
  if (!rc && ng > 0) {
    e = dev_malloc_async((void **)&Xg, sizeof(double) * (size_t)ng * d, s);
    if (e == hipSuccess) e = dev_malloc_async((void **)&Ag, sizeof(double) * (size_t)ng * k1, s);
    if (e != hipSuccess) rc = hip_fail(e, "mlp gate");
    if (!rc) {
      hipLaunchKernelGGL(k_gather_rows, dim3(grid_of((int64_t)ng * d)), dim3(256), 0, s, X, idx, (int64_t)ng, d, Xg);
      rc = hdmr_eval(route->served_full, Xg, (int64_t)ng, Ag, k1, precision, s);
      if (!rc)
        hipLaunchKernelGGL(k_scatter_rows, dim3(grid_of((int64_t)ng * k1)), dim3(256), 0, s, Ag, idx, (int64_t)ng, k1,
                           route->d_mlp_cols, m, Y);
    }
  }
  const_cast<mlp_route *>(route)->last_gated = (int64_t)ng;
  (void)hipFreeAsync(P2, s);
  (void)hipFreeAsync(idx, s);
  (void)hipFreeAsync(Xg, s);
  (void)hipFreeAsync(Ag, s);
  return rc;
}

int mlp_route_set_gate(mlp_route *route, mlp_model *second, const hdmr_model *full, double tau) {
  clear_error();
  if (!route || !full || !(tau >= 0.0)) return fail(HDMR_EINVAL, "mlp_route_set_gate: bad argument");
  if (second && (second->d != route->d || second->m != route->m))
    return fail(HDMR_EINVAL, "mlp_route_set_gate: the second network's d or m differ");
  if (full->m != route->m || full->d != route->d) return fail(HDMR_EINVAL, "mlp_route_set_gate: model d or m differ");
  int rc = set_device(route->net);
  if (rc) return rc;
  if (route->served_full) {
    hdmr_free(route->served_full);
    route->served_full = nullptr;
  }
  route->second = nullptr;
  if (!second) return HDMR_OK;  // gate off
  if (!route->mlp_cols.empty() &&
      (rc = hdmr_model_select(full, 0, nullptr, (int32_t)route->mlp_cols.size(), route->mlp_cols.data(), 1,
                              &route->served_full)))
    return rc;
  if (!route->d_gate_count) HDMR_HIP(dev_malloc((void **)&route->d_gate_count, sizeof(unsigned long long)));
  route->second = second;
  route->gate_tau = tau;
  return HDMR_OK;
}

int mlp_route_gated(const mlp_route *route, int64_t *n_gated) {
  clear_error();
  if (!route || !n_gated) return fail(HDMR_EINVAL, "mlp_route_gated: null argument");
  *n_gated = route->last_gated;
  return HDMR_OK;
}

int mlp_eval_routed(const mlp_route *route, const double *X, int64_t n, double *Y, int32_t precision,
                    hdmr_stream_t stream) {
  clear_error();
  if (!route || n < 0 || (n > 0 && (!X || !Y))) return fail(HDMR_EINVAL, "mlp_eval_routed: bad argument");
  if (check_ptr(X) || check_ptr(Y)) return HDMR_EINVAL;
  if (n == 0) return HDMR_OK;
  int rc = set_device(route->net);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int32_t m = route->m;
  const int32_t k1 = (int32_t)route->mlp_cols.size(), kf = (int32_t)route->fb_cols.size();
  double *P = nullptr, *A = nullptr, *B = nullptr;
  hipError_t e = hipSuccess;
  if (k1 > 0) {
    e = dev_malloc_async((void **)&P, sizeof(double) * (size_t)n * m, s);
    if (e == hipSuccess) e = dev_malloc_async((void **)&A, sizeof(double) * (size_t)n * k1, s);
  }
  if (e == hipSuccess && kf > 0) e = dev_malloc_async((void **)&B, sizeof(double) * (size_t)n * kf, s);
  if (e != hipSuccess) {
    rc = hip_fail(e, "mlp_eval_routed");
  } else {
    if (k1 > 0 && !(rc = forward_rows(route->net, X, n, P, s)) &&
        !(rc = hdmr_eval(route->order1, X, n, A, k1, precision, stream)))
      hipLaunchKernelGGL(k_scatter_cols, dim3(grid_of(n * k1)), dim3(256), 0, s, A, k1, route->d_mlp_cols, P, n, m, Y);
    if (!rc && k1 > 0 && route->second) rc = gate_points(route, X, n, P, Y, precision, s);
    if (!rc && kf > 0 && !(rc = hdmr_eval(route->fallback, X, n, B, kf, precision, stream)))
      hipLaunchKernelGGL(k_scatter_cols, dim3(grid_of(n * kf)), dim3(256), 0, s, B, kf, route->d_fb_cols,
                         (const double *)nullptr, n, m, Y);
    if (!rc && (e = hipGetLastError()) != hipSuccess) rc = hip_fail(e, "mlp_eval_routed");
  }
  (void)hipFreeAsync(P, s);
  (void)hipFreeAsync(A, s);
  (void)hipFreeAsync(B, s);
  return rc;
}

void mlp_route_free(mlp_route *route) {
  if (!route) return;
  (void)hipDeviceSynchronize();
  delete route;
}

}  // extern "C"
