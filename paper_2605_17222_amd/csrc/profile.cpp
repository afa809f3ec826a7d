// Per-kernel timing for benchmarks: when a kernel's bit is enabled, each of its
// launches is bracketed by two HIP events recorded on the launch stream, and
// the launch's algorithmic bytes are accumulated beside them.
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace ckks {

namespace {

struct Rec {
  int id;
  hipEvent_t a, b;
  double bytes;
};

std::mutex g_mu;
int g_mask = 0;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void recycle_all() {
  for (Rec& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
}

}  // namespace

ProfScope::ProfScope(int id, hipStream_t s, double bytes) : id_(id), s_(s), bytes_(bytes) {
  if (!(g_mask & (1 << id))) return;
  std::lock_guard<std::mutex> lk(g_mu);
  a_ = take();
  b_ = take();
  if (a_ && b_ && hipEventRecord((hipEvent_t)a_, s) == hipSuccess) active_ = true;
}

ProfScope::~ProfScope() {
  if (!active_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (hipEventRecord((hipEvent_t)b_, s_) == hipSuccess)
    g_recs.push_back(Rec{id_, (hipEvent_t)a_, (hipEvent_t)b_, bytes_});
}

}  // namespace ckks

extern "C" {

int ckks_profile_enable(int mask) {
  std::lock_guard<std::mutex> lk(ckks::g_mu);
  for (auto& r : ckks::g_recs) {
    (void)hipEventSynchronize(r.b);
  }
  ckks::recycle_all();
  ckks::g_mask = mask;
  return CKKS_OK;
}

int ckks_profile_read(int kernel, int* launches, double* total_ms, double* total_bytes) {
  if (kernel < 0 || kernel >= CKKS_KERNEL_COUNT || !launches || !total_ms || !total_bytes) return CKKS_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(ckks::g_mu);
  int n = 0;
  double ms = 0, bytes = 0;
  for (auto& r : ckks::g_recs) {
    if (r.id != kernel) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return CKKS_E_DEVICE;
    float t = 0;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return CKKS_E_DEVICE;
    ++n;
    ms += t;
    bytes += r.bytes;
  }
  *launches = n;
  *total_ms = ms;
  *total_bytes = bytes;
  return CKKS_OK;
}

}  // extern "C"
