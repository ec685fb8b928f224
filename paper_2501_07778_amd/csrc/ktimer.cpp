// ktimer.cpp — optional timing of chosen kernels with HIP events recorded
// on the stream each launch goes to (the events bracket the launch, so the
// elapsed time is that launch's device time on that stream).  Off unless a
// caller turns it on; events come from a reused pool.
#include <mutex>
#include <string>
#include <vector>

#include "step.h"

namespace qtt {
namespace {

struct Rec {
  int id;
  hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
size_t g_used = 0;

const char *const kNames[KT_COUNT] = {"k_svd_step", "k_sketch_qr", "k_qr_step"};

hipEvent_t take_event() {
  if (g_used == g_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_pool.push_back(e);
  }
  return g_pool[g_used++];
}

}  // namespace

int ktimer_begin(int id, hipStream_t s) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_on) return -1;
  Rec r{id, take_event(), take_event()};
  if (!r.a || !r.b || hipEventRecord(r.a, s) != hipSuccess) return -1;
  g_recs.push_back(r);
  return (int)g_recs.size() - 1;
}

bool ktimer_active() {
  std::lock_guard<std::mutex> g(g_mu);
  return g_on;
}

void ktimer_end(int handle, hipStream_t s) {
  if (handle < 0) return;
  std::lock_guard<std::mutex> g(g_mu);
  if (handle < (int)g_recs.size()) (void)hipEventRecord(g_recs[handle].b, s);
}

}  // namespace qtt

using namespace qtt;

extern "C" qtt_status qtt_kernel_timing(int32_t enable) {
  std::lock_guard<std::mutex> g(g_mu);
  g_recs.clear();
  g_used = 0;
  g_on = enable != 0;
  return QTT_OK;
}

extern "C" qtt_status qtt_kernel_timing_read(const char *kernel, double *ms, int64_t *launches) {
  if (!kernel || !ms || !launches) return fail(QTT_E_INVAL, "NULL argument");
  int id = -1;
  for (int i = 0; i < KT_COUNT; ++i)
    if (std::string(kernel) == kNames[i]) id = i;
  if (id < 0) return fail(QTT_E_INVAL, std::string("no timed kernel named ") + kernel);
  std::lock_guard<std::mutex> g(g_mu);
  double tot = 0.0;
  int64_t n = 0;
  for (const Rec &r : g_recs) {
    if (r.id != id) continue;
    hipError_t e = hipEventSynchronize(r.b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) return fail(QTT_E_HIP, std::string("event timing: ") + hipGetErrorString(e));
    tot += t;
    ++n;
  }
  *ms = tot;
  *launches = n;
  return QTT_OK;
}
