// Device timing of evaluation stages: event pairs recorded on the launch
// stream around each stage, resolved on read.
#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "hdmr_internal.h"

namespace hdmr {
namespace {

struct Record {
  int stage;
  hipEvent_t start, stop;
};

std::mutex g_mu;
std::atomic<bool> g_on{false};
std::vector<Record> g_records;

void discard_locked() {
  for (Record &r : g_records) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  g_records.clear();
}

}  // namespace

bool timing_on() { return g_on.load(std::memory_order_relaxed); }

StageTimer::StageTimer(int st, hipStream_t s) : stage(st), stream(s) {
  if (!timing_on()) return;
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return;
  if (hipEventRecord(e, stream) != hipSuccess) {
    (void)hipEventDestroy(e);
    return;
  }
  start = e;
}

StageTimer::~StageTimer() {
  if (!start) return;
  hipEvent_t stop = nullptr;
  if (hipEventCreate(&stop) != hipSuccess || hipEventRecord(stop, stream) != hipSuccess) {
    if (stop) (void)hipEventDestroy(stop);
    (void)hipEventDestroy((hipEvent_t)start);
    return;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_records.push_back(Record{stage, (hipEvent_t)start, stop});
}

}  // namespace hdmr

using namespace hdmr;

extern "C" {

int hdmr_timing_enable(int32_t on) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  discard_locked();
  g_on.store(on != 0);
  return HDMR_OK;
}

int hdmr_timing_read(const char *stage, double *total_ms, int64_t *launches) {
  clear_error();
  if (!stage || !total_ms || !launches) return fail(HDMR_EINVAL, "null argument");
  static const char *names[STAGE_COUNT] = {"sort", "rows", "contract"};
  int st = -1;
  for (int i = 0; i < STAGE_COUNT; ++i)
    if (std::strcmp(stage, names[i]) == 0) st = i;
  if (st < 0) return fail(HDMR_EINVAL, std::string("unknown stage '") + stage + "'");
  std::lock_guard<std::mutex> lk(g_mu);
  double sum = 0.0;
  int64_t cnt = 0;
  for (Record &r : g_records) {
    if (r.stage != st) continue;
    HDMR_HIP(hipEventSynchronize(r.stop));
    float ms = 0.f;
    HDMR_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
    sum += ms;
    ++cnt;
  }
  *total_ms = sum;
  *launches = cnt;
  return HDMR_OK;
}

}  // extern "C"
