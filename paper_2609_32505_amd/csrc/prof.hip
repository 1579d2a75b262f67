// Per-kernel-class launch timing: when enabled, every instrumented launch is
// bracketed by a pair of HIP events recorded on its own stream; reading the
// totals synchronises on the recorded events.
#include <mutex>
#include <new>
#include <vector>

#include "prof.hpp"
#include "svdp.h"

namespace {
struct Rec {
  int kind;
  hipEvent_t a, b;
  double work;
};
std::mutex g_mu;
bool g_on = false;
double* g_dev_work = nullptr;  // PROF_KINDS device counters, allocated on first enable
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

// phase scopes nest (a fallback rerun contains CANS and eigh phases): only
// the outermost one on a thread records
thread_local int t_phase_depth = 0;

ProfScope::ProfScope(int k, hipStream_t s, double work)
    : kind(k), st(s), slot(-1), phase(k >= PROF_PHASE_BOUND && k <= PROF_PHASE_QR) {
  if (phase && t_phase_depth++ > 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  hipEvent_t a = get_event(), b = get_event();
  if (!a || !b) return;
  if (hipEventRecord(a, st) != hipSuccess) return;
  g_recs.push_back({kind, a, b, work});
  slot = (int)g_recs.size() - 1;
}

ProfScope::~ProfScope() {
  if (phase) --t_phase_depth;
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (slot < (int)g_recs.size()) (void)hipEventRecord(g_recs[slot].b, st);
}

void ProfScope::next(int k) {
  const hipStream_t s = st;
  this->~ProfScope();
  new (this) ProfScope(k, s, 0.0);
}

double* prof_work_dev() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_on ? g_dev_work : nullptr;
}

extern "C" {

void svdp_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (on && !g_dev_work) {
    if (hipMalloc((void**)&g_dev_work, PROF_KINDS * sizeof(double)) != hipSuccess) g_dev_work = nullptr;
    else (void)hipMemset(g_dev_work, 0, PROF_KINDS * sizeof(double));
  }
  g_on = on != 0;
}

void svdp_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  if (g_dev_work) {
    (void)hipDeviceSynchronize();
    (void)hipMemset(g_dev_work, 0, PROF_KINDS * sizeof(double));
  }
}

int svdp_profile_read(int kind, double* total_ms, int64_t* launches, double* work) {
  std::lock_guard<std::mutex> lk(g_mu);
  double t = 0.0, wk = 0.0;
  int64_t c = 0;
  for (auto& r : g_recs) {
    if (r.kind != kind) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return SVDP_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return SVDP_ERR_HIP;
    t += ms;
    wk += r.work;
    ++c;
  }
  if (g_dev_work && kind >= 0 && kind < PROF_KINDS) {
    double dw = 0.0;
    if (hipDeviceSynchronize() != hipSuccess) return SVDP_ERR_HIP;
    if (hipMemcpy(&dw, g_dev_work + kind, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return SVDP_ERR_HIP;
    wk += dw;
  }
  if (total_ms) *total_ms = t;
  if (launches) *launches = c;
  if (work) *work = wk;
  return SVDP_OK;
}

}  // extern "C"
