// Optional per-step timing of the apply (bfly_timing_enable/read): HIP
// events recorded around kernel launches on the launching stream.
#include <mutex>
#include <vector>

#include "bfly_internal.h"

namespace bfly {
namespace {

struct Pending {
  int kind, stages, inits, switches;
  hipEvent_t b, e;
};

struct State {
  std::mutex mu;
  bool on = false;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double ms[kNumSteps] = {};
  int64_t launches[kNumSteps] = {}, stages[kNumSteps] = {}, inits[kNumSteps] = {}, switches[kNumSteps] = {};
  std::vector<LaunchRecord> log;  // the launches the last timing_read collected, in order
};

State& st() {
  static State s;
  return s;
}

hipEvent_t take(State& s) {
  if (!s.pool.empty()) {
    hipEvent_t e = s.pool.back();
    s.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

bool timing_on() { return st().on; }

void timing_set(bool on) {
  State& s = st();
  std::lock_guard<std::mutex> lk(s.mu);
  s.on = on;
}

StepTimer::StepTimer(int kind, hipStream_t s, int stages, int inits, int switches)
    : kind_(kind), stages_(stages), inits_(inits), switches_(switches), s_(s) {
  State& S = st();
  if (!S.on) return;
  std::lock_guard<std::mutex> lk(S.mu);
  b_ = take(S);
  if (b_) (void)hipEventRecord(b_, s_);
}

StepTimer::~StepTimer() {
  if (!b_) return;
  State& S = st();
  std::lock_guard<std::mutex> lk(S.mu);
  hipEvent_t e = take(S);
  if (!e) {
    S.pool.push_back(b_);
    return;
  }
  (void)hipEventRecord(e, s_);
  S.pending.push_back({kind_, stages_, inits_, switches_, b_, e});
}

hipError_t timing_read(double* ms, int64_t* launches, int64_t* stages, int64_t* inits, int64_t* switches) {
  State& S = st();
  std::lock_guard<std::mutex> lk(S.mu);
  hipError_t err = hipSuccess;
  S.log.clear();
  for (const Pending& p : S.pending) {
    hipError_t e = hipEventSynchronize(p.e);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, p.b, p.e);
    if (e != hipSuccess) {
      err = e;
    } else {
      S.ms[p.kind] += t;
      S.launches[p.kind] += 1;
      S.stages[p.kind] += p.stages;
      S.inits[p.kind] += p.inits;
      S.switches[p.kind] += p.switches;
      S.log.push_back({p.kind, p.stages, p.inits, p.switches, (double)t});
    }
    S.pool.push_back(p.b);
    S.pool.push_back(p.e);
  }
  S.pending.clear();
  for (int k = 0; k < kNumSteps; ++k) {
    ms[k] = S.ms[k];
    launches[k] = S.launches[k];
    stages[k] = S.stages[k];
    inits[k] = S.inits[k];
    switches[k] = S.switches[k];
    S.ms[k] = 0;
    S.launches[k] = S.stages[k] = S.inits[k] = S.switches[k] = 0;
  }
  return err;
}

int timing_launches(int cap, LaunchRecord* out) {
  State& S = st();
  std::lock_guard<std::mutex> lk(S.mu);
  const int n = (int)S.log.size();
  for (int i = 0; i < n && i < cap; ++i) out[i] = S.log[i];
  return n;
}

}  // namespace bfly
