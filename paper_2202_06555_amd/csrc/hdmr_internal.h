// Internal declarations shared by the host and device sources of libhdmr.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hdmr.h"

namespace hdmr {

constexpr int KMAX = 4;        // largest |S| a component may have
constexpr int MAX_LEVEL = 30;  // largest level per dimension

// How the row of the active cell of a level multi-index is found.
enum TupKind : uint8_t {
  TUP_FULL = 0,   // every cell stored: row = row_base + slot
  TUP_DENSE = 1,  // int32 slot table at tab[aux .. aux + ncells): row or -1
  TUP_HASH = 2,   // open addressing at tab[aux .. aux + 2*(mask+1)): (slot, row) pairs
};

// One stored level multi-index l of one component ("tuple").  Its rows are
// contiguous and sorted by slot, the mixed-radix number of the cell
// (c_q = (i_q - 1) / 2 per dimension, last dimension fastest).
struct alignas(16) TupDesc {
  double w;          // weight w_S of the owning component
  int32_t row_base;  // first row of the tuple
  int32_t aux;       // table offset (DENSE, HASH)
  int32_t mask;      // hash capacity - 1 (HASH)
  int32_t comp;      // owning component
  int16_t dims[KMAX];
  uint8_t lv[KMAX];
  uint8_t k, kind, lsum, pad_;
};
static_assert(sizeof(TupDesc) == 48, "TupDesc layout");

// Device view of a model (passed to kernels by value).
struct ModelView {
  const TupDesc *tups;
  const int32_t *tab;
  const double *alpha;   // n_rows x ms, FP64 (row stride ms = m rounded up to even)
  const double *c0;      // m
  const int32_t *comp_tup;  // n_components + 1: tuple ranges per component
  int32_t ntup, ncomp, d, m, ms;
};

// One sorted evaluation pass: points are ordered by their cell in the key
// dimensions (cell_lv[q] levels of dims[q]); the listed components (whose
// dimensions are a subset of the key) are evaluated together.
constexpr int PASS_MAX_COMPS = 8;
struct Pass {
  int32_t k;
  int32_t dims[KMAX];
  int32_t cell_lv[KMAX];
  int32_t shift[KMAX];
  int32_t key_bits;
  int32_t tup_begin, tup_end;  // range in the pass-tuple list
  int64_t list_bound;          // (cell, row) incidences summed over all cells
};
// A tuple as seen from a pass: key position of each of its dimensions.
struct alignas(8) PassTup {
  int32_t tup;
  uint8_t pos[KMAX];
};

struct Component {
  int32_t k;
  int32_t dims[KMAX];
  double w;
  int64_t row_begin, row_end;    // global rows
  int32_t tup_begin, tup_end;    // global tuples
};

// One candidate index set of the adaptive build (Alg. 2): eta of eq (3.19)
// (NaN when not tested) and whether it was kept.
struct DdsgCandidate {
  int32_t k;
  int32_t dims[KMAX];
  double eta;
  uint8_t kept;
};

}  // namespace hdmr

struct hdmr_model {
  int device = 0;
  int32_t d = 0, m = 0, ms = 0;
  int64_t n_rows = 0;
  int32_t max_level = 0, max_k = 0;
  std::vector<hdmr::Component> comps;
  std::vector<hdmr::TupDesc> tups_h;
  // host copies in internal row order (export, rebuilds)
  std::vector<uint8_t> lv_h;     // n_rows x KMAX
  std::vector<uint32_t> ix_h;    // n_rows x KMAX
  std::vector<double> c0_h;
  // device buffers (owned)
  hdmr::TupDesc *tups = nullptr;
  int32_t *tab = nullptr;
  double *alpha = nullptr;
  float *alpha32 = nullptr;   // FP32 copy of alpha (same layout) for the mixed path
  double *c0 = nullptr;
  int32_t *comp_tup = nullptr;
  int64_t tab_entries = 0;
  int64_t device_bytes = 0;
  // sorted-evaluation plan
  std::vector<hdmr::Pass> passes;
  std::vector<hdmr::PassTup> pass_tups_h;
  hdmr::PassTup *pass_tups = nullptr;
  int32_t max_pass_tups = 0;
  // adaptive-build report (Alg. 2): candidates in build order, rho per order
  std::vector<hdmr::DdsgCandidate> ddsg;
  std::vector<double> ddsg_rho;

  hdmr::ModelView view() const {
    return hdmr::ModelView{tups, tab, alpha, c0, comp_tup, (int32_t)tups_h.size(), (int32_t)comps.size(), d, m, ms};
  }
};

namespace hdmr {

// thread-local error message + status helpers
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// Every device allocation of the library goes through these two (model.hip).
// For error-path tests a failure can be forced from the host: with the
// environment variable HDMR_FAIL_ALLOC=k (k >= 0), the allocation numbered k
// (from 0, counted since the variable last changed value) returns
// hipErrorOutOfMemory without allocating.
hipError_t dev_malloc(void **p, size_t bytes);
hipError_t dev_malloc_async(void **p, size_t bytes, hipStream_t s);
void clear_error();

#define HDMR_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hdmr::hip_fail(e_, #call); \
  } while (0)

// Construct the device model from host rows (defined in model.hip).
struct HostComponent {
  int32_t k;
  int32_t dims[KMAX];
  double w;
  int64_t n;
  const uint8_t *lv;    // n x k
  const uint32_t *ix;   // n x k
  const double *alpha;  // n x m (host), or NULL when src_rows is given
  const int64_t *src_rows;  // n rows of a device source matrix (see DeviceAlphaSource)
};
// Surpluses already on the device: row r of component c is
// src[c.src_rows[r] * stride + col .. + m).
struct DeviceAlphaSource {
  const double *src;
  int32_t stride, col;
};
int make_model(int32_t d, int32_t m, const double *c0, const std::vector<HostComponent> &comps, hdmr_model **out,
               const DeviceAlphaSource *dsrc = nullptr);

int set_device_of(const hdmr_model *model);
void keep_pool_memory(int device);

// Cell-sorted evaluation (eval_sorted.hip), precision HDMR_PLAIN_FP64 or
// HDMR_MIXED; variant selects the contraction's tile shape (bit 0: the
// smaller row batch; bit 1: work items of half the points; bit 2: a
// persistent grid of three workgroups per CU; bit 3: one of two per CU), 0
// is the default.  With G (n x d x m, plain precision only) the
// gradient is computed as well.
// ws_base (device, ws_bytes bytes) supplies the workspace; with NULL it is
// allocated stream-ordered on the device's pool and released at the end.
// events (8, optional): persistent events to use instead of per-call ones.
int eval_sorted(const hdmr_model *model, const double *X, int64_t n, double *F, int precision, hipStream_t stream,
                int variant = 0, double *G = nullptr, void *ws_base = nullptr, size_t ws_bytes = 0,
                hipEvent_t *events = nullptr);
// Workspace bytes eval_sorted needs for n points at that precision.
int eval_sorted_workspace(const hdmr_model *model, int64_t n, int precision, size_t *bytes);

// The static workspace of hdmr_eval_noalloc on a device (eval_sorted.hip):
// set-up once per device with that device current (address of the device
// array, the second stream, persistent events), then its address and size.
int noalloc_setup(int device);
int noalloc_workspace(int device, void **ptr, size_t *bytes, hipEvent_t **events);

// Drop every cached batched-launch graph that refers to the model (batched.hip).
void batched_forget(const hdmr_model *model);

// Plan the sorted-evaluation passes of a model and upload the pass tuples.
int plan_passes(hdmr_model *M);

// Device timing of evaluation stages (timing.hip).
enum TimedStage : int { STAGE_SORT = 0, STAGE_ROWS = 1, STAGE_CONTRACT = 2, STAGE_COUNT = 3 };
bool timing_on();
// Records a start event on construction and a stop event on destruction
// when timing is enabled; does nothing otherwise.
struct StageTimer {
  StageTimer(int stage, hipStream_t s);
  ~StageTimer();
  StageTimer(const StageTimer &) = delete;
  StageTimer &operator=(const StageTimer &) = delete;
  int stage;
  hipStream_t stream;
  void *start = nullptr;
};

}  // namespace hdmr

namespace hdmr {

// Slot hash of HASH tuples (integer finaliser; host and device agree).
__host__ __device__ inline uint32_t slot_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

constexpr uint32_t HASH_EMPTY = 0xFFFFFFFFu;

}  // namespace hdmr
