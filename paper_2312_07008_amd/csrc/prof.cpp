// Opt-in stage timers: HIP events recorded around the library's own launches
// on the caller's stream, accumulated when the entry point synchronizes.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/dfpt2.h"
#include "host.h"

namespace dfpt2 {

namespace {
struct Pending {
  int stage;
  hipEvent_t a, b;
};
struct Profiler {
  bool on = false;
  double ms[DFPT2_NSTAGE] = {};
  int64_t launches[DFPT2_NSTAGE] = {};
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
};
// one set of counters per host thread: a pass is timed by the thread that issues it,
// and threads that run passes concurrently do not see each other's stages
thread_local Profiler g_prof;

hipEvent_t get_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

ProfScope::ProfScope(int stage, hipStream_t s) : stage_(stage), s_(s), a_(nullptr) {
  if (!g_prof.on || stage < 0) return;
  a_ = get_event();
  if (a_ && hipEventRecord(a_, s_) != hipSuccess) a_ = nullptr;
}

void ProfScope::close() {
  if (!a_) return;
  hipEvent_t a = a_;
  a_ = nullptr;
  hipEvent_t b = get_event();
  if (!b || hipEventRecord(b, s_) != hipSuccess) {
    g_prof.pool.push_back(a);
    return;
  }
  g_prof.pending.push_back(Pending{stage_, a, b});
}

void prof_flush() {
  for (const Pending& p : g_prof.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_prof.ms[p.stage] += ms;
      g_prof.launches[p.stage] += 1;
    }
    g_prof.pool.push_back(p.a);
    g_prof.pool.push_back(p.b);
  }
  g_prof.pending.clear();
}

}  // namespace dfpt2

using namespace dfpt2;

extern "C" {

int dfpt2_profile_enable(int on) {
  prof_flush();
  g_prof.on = (on != 0);
  for (int i = 0; i < DFPT2_NSTAGE; ++i) {
    g_prof.ms[i] = 0.0;
    g_prof.launches[i] = 0;
  }
  return DFPT2_OK;
}

int dfpt2_profile_read(double* ms, int64_t* launches) {
  prof_flush();
  for (int i = 0; i < DFPT2_NSTAGE; ++i) {
    if (ms) ms[i] = g_prof.ms[i];
    if (launches) launches[i] = g_prof.launches[i];
  }
  return DFPT2_OK;
}

}  // extern "C"
