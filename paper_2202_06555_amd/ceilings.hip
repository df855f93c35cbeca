// Measured ceilings of one gfx950 device, the denominators of the
// multi-ceiling roofline that bench.py reports for the evaluation kernels:
//   copy      : streaming HBM read + write (16-byte vector accesses);
//   rmw       : read-modify-write of randomly ordered output rows, the access
//               pattern of the contraction's output update (row widths and
//               layouts as the kernels use them, buffer sizes from beyond
//               the 256 MB last-level cache down to a few MB);
//   mfma_f64  : v_mfma_f64_16x16x4f64 from registers;
//   mfma_bf16 : v_mfma_f32_16x16x32_bf16 from registers;
//   valu_f64  : FP64 FMA chains;
//   lds_gather: 8-byte LDS reads at lane-scattered addresses.
// Every probe prints one JSON line.  Each kernel's indexing stays inside its
// buffers by construction (bounds are checked on the host before launch).
//
//   bench_ceilings [probe ...]     (no argument: every probe)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#define CK(call)                                                                          \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      std::fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));              \
      std::exit(1);                                                                       \
    }                                                                                     \
  } while (0)

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__global__ void k_copy(const double4 *__restrict__ a, double4 *__restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// Output rows visited in the order of perm (a permutation of [0, nrows)):
// a wave takes 16 rows per step; lane (kk = lane / 16, jj = lane % 16) holds
// rows kk + 4 i (i < 4) and the columns jj + 16 c (c < width / 16 rounded up),
// as the contraction's accumulators are laid out.  Row r, column o lives at
// F[r * stride + o] (row-major) or, with colblock, at F[(o / 16) * nrows * 16
// + r * 16 + o % 16] (16-column blocks of 128 bytes).  Each element gets
// +1.0, so after reps visits every element equals reps.
__global__ __launch_bounds__(256) void k_rmw(double *__restrict__ F, const int32_t *__restrict__ perm, int64_t nrows,
                                             int stride, int width, int colblock) {
  const int lane = threadIdx.x & 63, kk = lane >> 4, jj = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int ncb = (width + 15) / 16;
  for (int64_t base = wave * 16; base < nrows; base += nw * 16) {
    for (int c = 0; c < ncb; ++c) {
      const int o = 16 * c + jj;
      double f[4];
      int64_t at[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t e = base + kk + 4 * i;
        const int64_t r = e < nrows ? perm[e] : 0;
        at[i] = colblock ? (int64_t)c * nrows * 16 + r * 16 + jj : r * stride + o;
        f[i] = (e < nrows && o < width) ? F[at[i]] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t e = base + kk + 4 * i;
        if (e < nrows && o < width) F[at[i]] = f[i] + 1.0;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_mfma_f64(double *__restrict__ out, int iters) {
  v4d acc[4];
  for (int j = 0; j < 4; ++j) acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
  double a = 1.0 + threadIdx.x * 1e-9, b = 1.0 - threadIdx.x * 1e-9;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
  }
  double s = 0.0;
  for (int j = 0; j < 4; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mfma_bf16(float *__restrict__ out, int iters) {
  v4f acc[4];
  for (int j = 0; j < 4; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
  bf16x8 a, b;
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1.0f + e * 1e-3f);
    b[e] = (__bf16)(1.0f - e * 1e-3f);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
  }
  float s = 0.f;
  for (int j = 0; j < 4; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_valu_f64(double *__restrict__ out, int iters) {
  double x[8];
  for (int j = 0; j < 8; ++j) x[j] = 1.0 + (threadIdx.x + j) * 1e-12;
  const double a = 0.999999, b = 1e-7;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = fma(x[j], a, b);
  }
  double s = 0.0;
  for (int j = 0; j < 8; ++j) s += x[j];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 8-byte LDS reads: lane l of step i reads element (l * 37 + i * 13) mod 8192
// of a 64 KB array (scattered over the banks).
__global__ __launch_bounds__(256) void k_lds_gather(double *__restrict__ out, int iters) {
  __shared__ double s[8192];
  for (int i = threadIdx.x; i < 8192; i += blockDim.x) s[i] = (double)i;
  __syncthreads();
  double acc = 0.0;
  const int l = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += s[(l * 37 + (it * 8 + u) * 13) & 8191];
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

struct Timer {
  hipEvent_t a, b;
  Timer() {
    CK(hipEventCreate(&a));
    CK(hipEventCreate(&b));
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  void start() { CK(hipEventRecord(a, 0)); }
  double stop_ms() {
    CK(hipEventRecord(b, 0));
    CK(hipEventSynchronize(b));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
};

int num_cus() {
  hipDeviceProp_t p;
  CK(hipGetDeviceProperties(&p, 0));
  return p.multiProcessorCount;
}

void probe_copy() {
  const int64_t bytes = 2LL << 30;  // 2 GiB each way
  const int64_t n4 = bytes / 32;
  double4 *a = nullptr, *b = nullptr;
  CK(hipMalloc((void **)&a, bytes));
  CK(hipMalloc((void **)&b, bytes));
  CK(hipMemset(a, 0, bytes));
  const int grid = num_cus() * 16;
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, 0, a, b, n4);
  Timer t;
  const int reps = 10;
  t.start();
  for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, 0, a, b, n4);
  const double ms = t.stop_ms() / reps;
  std::printf("{\"probe\": \"copy\", \"bytes_per_launch\": %lld, \"ms\": %.4f, \"GBps\": %.1f}\n",
              (long long)(2 * bytes), ms, 2.0 * bytes / ms / 1e6);
  CK(hipFree(a));
  CK(hipFree(b));
}

void probe_rmw() {
  const int64_t sizes[] = {4000000, 2000000, 1000000, 500000, 250000, 100000, 20000};
  struct Layout {
    const char *name;
    int stride, width, colblock;
  } layouts[] = {{"rowmajor_m51", 51, 51, 0},   {"rowmajor_pad64", 64, 64, 0}, {"colblock16_m64", 16, 64, 1},
                 {"rowmajor_pad56", 56, 56, 0}, {"rowmajor_pad48", 48, 48, 0}};
  const int64_t max_rows = sizes[0];
  double *F = nullptr;
  int32_t *perm_d = nullptr;
  CK(hipMalloc((void **)&F, (size_t)max_rows * 64 * sizeof(double)));
  CK(hipMalloc((void **)&perm_d, (size_t)max_rows * sizeof(int32_t)));
  std::mt19937_64 rng(12345);
  const int grid = num_cus() * 12;
  for (int64_t nrows : sizes) {
    std::vector<int32_t> perm(nrows);
    for (int64_t i = 0; i < nrows; ++i) perm[i] = (int32_t)i;
    std::shuffle(perm.begin(), perm.end(), rng);
    CK(hipMemcpy(perm_d, perm.data(), nrows * sizeof(int32_t), hipMemcpyHostToDevice));
    for (const Layout &L : layouts) {
      // bounds: row-major touches r * stride + o < nrows * stride (o < width <= stride);
      // column blocks touch c * nrows * 16 + r * 16 + jj < ceil(width / 16) * nrows * 16
      const int64_t span = L.colblock ? (int64_t)((L.width + 15) / 16) * nrows * 16 : nrows * L.stride;
      if (span > max_rows * 64 || (!L.colblock && L.width > L.stride)) std::abort();
      CK(hipMemset(F, 0, (size_t)span * sizeof(double)));
      hipLaunchKernelGGL(k_rmw, dim3(grid), dim3(256), 0, 0, F, perm_d, nrows, L.stride, L.width, L.colblock);
      // enough visits for about 40 ms of work
      const int reps = (int)std::max<int64_t>(4, std::min<int64_t>(400, 40 * 4000000 / (nrows * 2) / 4));
      Timer t;
      t.start();
      for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_rmw, dim3(grid), dim3(256), 0, 0, F, perm_d, nrows, L.stride, L.width, L.colblock);
      const double ms = t.stop_ms() / reps;
      // check: every element visited reps + 1 times
      double probe_v = 0.0;
      CK(hipMemcpy(&probe_v, F, sizeof(double), hipMemcpyDeviceToHost));
      const double useful = 2.0 * nrows * L.width * 8.0;
      std::printf("{\"probe\": \"rmw\", \"layout\": \"%s\", \"rows\": %lld, \"footprint_MB\": %.1f, \"ms\": %.4f, "
                  "\"useful_GBps\": %.1f, \"rows_per_us\": %.1f, \"check\": %.0f}\n",
                  L.name, (long long)nrows, span * 8.0 / 1e6, ms, useful / ms / 1e6, nrows / ms / 1e3, probe_v);
      std::fflush(stdout);
    }
  }
  CK(hipFree(F));
  CK(hipFree(perm_d));
}

template <typename K, typename T>
void probe_alu(const char *name, K kern, double flops_per_wave_iter, int iters) {
  const int grid = num_cus() * 8;
  T *out = nullptr;
  CK(hipMalloc((void **)&out, (size_t)grid * 256 * sizeof(T)));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, 0, out, 16);
  Timer t;
  t.start();
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, 0, out, iters);
  const double ms = t.stop_ms();
  const double flops = flops_per_wave_iter * iters * (grid * 4.0);
  std::printf("{\"probe\": \"%s\", \"ms\": %.4f, \"TFLOPs\": %.2f}\n", name, ms, flops / ms / 1e9);
  CK(hipFree(out));
}

void probe_lds() {
  const int grid = num_cus() * 8, iters = 4096;
  double *out = nullptr;
  CK(hipMalloc((void **)&out, (size_t)grid * 256 * sizeof(double)));
  hipLaunchKernelGGL(k_lds_gather, dim3(grid), dim3(256), 0, 0, out, 16);
  Timer t;
  t.start();
  hipLaunchKernelGGL(k_lds_gather, dim3(grid), dim3(256), 0, 0, out, iters);
  const double ms = t.stop_ms();
  const double bytes = 8.0 * 8 * iters * grid * 256.0;
  std::printf("{\"probe\": \"lds_gather\", \"ms\": %.4f, \"TBps\": %.2f}\n", ms, bytes / ms / 1e9);
  CK(hipFree(out));
}

}  // namespace

int main(int argc, char **argv) {
  std::vector<std::string> want;
  for (int i = 1; i < argc; ++i) want.push_back(argv[i]);
  auto on = [&](const char *p) { return want.empty() || std::find(want.begin(), want.end(), p) != want.end(); };
  if (on("copy")) probe_copy();
  if (on("mfma_f64")) probe_alu<decltype(&k_mfma_f64), double>("mfma_f64", k_mfma_f64, 4 * 2.0 * 16 * 16 * 4, 20000);
  if (on("mfma_bf16"))
    probe_alu<decltype(&k_mfma_bf16), float>("mfma_bf16", k_mfma_bf16, 4 * 2.0 * 16 * 16 * 32, 20000);
  if (on("valu_f64")) probe_alu<decltype(&k_valu_f64), double>("valu_f64", k_valu_f64, 64 * 8 * 2.0, 20000);
  if (on("lds_gather")) probe_lds();
  if (on("rmw")) probe_rmw();
  return 0;
}
