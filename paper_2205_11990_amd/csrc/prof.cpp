#include "prof.hpp"

#include <mutex>
#include <vector>

namespace mpsv {

namespace {
struct Rec {
  int cls;
  double flops, bytes;
  bool nested;
};
thread_local int t_nested = 0;
std::mutex g_mu;
bool g_on = false;
std::vector<hipEvent_t> g_ev;  // pairs: 2*slot, 2*slot+1
std::vector<Rec> g_rec;
size_t g_used = 0;
}  // namespace

bool prof_enabled() { return g_on; }

void prof_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on;
  if (on) {
    g_used = 0;
    g_rec.clear();
  }
}

int prof_begin(hipStream_t s) {
  if (!g_on) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  if (2 * (g_used + 1) > g_ev.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      MPSV_HIP(hipEventCreate(&e));
      g_ev.push_back(e);
    }
  }
  const int slot = (int)g_used++;
  g_rec.push_back(Rec{kClsOther, 0.0, 0.0, false});
  MPSV_HIP(hipEventRecord(g_ev[2 * slot], s));
  return slot;
}

void prof_end(hipStream_t s, int slot, int cls, double flops, double bytes) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  MPSV_HIP(hipEventRecord(g_ev[2 * slot + 1], s));
  // a launch over lock-step instances does the work of each of them
  const double n = (double)inst_count();
  g_rec[slot] = Rec{cls, flops * n, bytes * n, t_nested > 0};
}

ProfNested::ProfNested() { ++t_nested; }
ProfNested::~ProfNested() { --t_nested; }

double prof_nested_flops(int cls) {
  MPSV_HIP(hipDeviceSynchronize());
  std::lock_guard<std::mutex> lk(g_mu);
  double f = 0.0;
  for (size_t i = 0; i < g_used; ++i)
    if (g_rec[i].cls == cls && g_rec[i].nested) f += g_rec[i].flops;
  return f;
}

void prof_read(int cls, long* launches, double* ms, double* flops,
               double* bytes) {
  MPSV_HIP(hipDeviceSynchronize());
  std::lock_guard<std::mutex> lk(g_mu);
  long n = 0;
  double t = 0, f = 0, b = 0;
  for (size_t i = 0; i < g_used; ++i) {
    if (g_rec[i].cls != cls) continue;
    float e = 0.0f;
    MPSV_HIP(hipEventElapsedTime(&e, g_ev[2 * i], g_ev[2 * i + 1]));
    ++n;
    t += e;
    f += g_rec[i].flops;
    b += g_rec[i].bytes;
  }
  if (launches) *launches = n;
  if (ms) *ms = t;
  if (flops) *flops = f;
  if (bytes) *bytes = b;
}

}  // namespace mpsv
