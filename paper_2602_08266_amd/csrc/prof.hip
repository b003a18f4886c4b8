// prof.hip -- optional per-kernel timing with HIP events on the launch stream.
//
// When enabled, every kernel launch of the library is bracketed by two events recorded on
// the stream it is launched on; reading the profile synchronises the events and returns the
// total duration and launch count per kernel class. Disabled, the bracket costs one branch.
#include <mutex>
#include <vector>

#include "common.hpp"

namespace ngs {
namespace {

struct Rec {
  int id;
  hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
int g_only = -1;  // >= 0: only this kernel class is timed
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
double g_ms[kProfKernels];
int64_t g_cnt[kProfKernels];

const char* const kNames[kProfKernels] = {
    "prepare_scene", "project", "depth_sort_hist", "depth_sort_scan", "depth_sort_scatter", "count_scan",
    "unused_emit", "unused_ranges", "tile_keys64", "render", "ig_back", "ig_finalize", "hessian_logdet",
    "score_combine", "fill", "tile_part_hist", "tile_part_scan", "tile_part_scatter", "ig_assign", "bwd_tiles", "bwd_params", "sur_gemm", "sur_forward",
    "sur_backward", "ig_front"};

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

void drain_locked() {
  for (Rec& r : g_recs) {
    float ms = 0.f;
    if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      g_ms[r.id] += ms;
      g_cnt[r.id] += 1;
    }
    if (r.a) g_pool.push_back(r.a);
    if (r.b) g_pool.push_back(r.b);
  }
  g_recs.clear();
}

}  // namespace

ProfScope::ProfScope(int id, hipStream_t st) : id_(id), st_(st), a_(nullptr) {
  if (!g_on || (g_only >= 0 && id != g_only)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t a = get_event();
  if (a) (void)hipEventRecord(a, st_);
  a_ = a;
}

ProfScope::~ProfScope() {
  if (!a_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t b = get_event();
  if (b) (void)hipEventRecord(b, st_);
  g_recs.push_back({id_, static_cast<hipEvent_t>(a_), b});
  if (g_recs.size() > 65536) drain_locked();
}

void prof_enable(bool on, int only) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  for (int i = 0; i < kProfKernels; ++i) { g_ms[i] = 0.0; g_cnt[i] = 0; }
  g_on = on;
  g_only = only;
}

bool prof_suspend() {
  std::lock_guard<std::mutex> lk(g_mu);
  const bool was = g_on;
  g_on = false;
  return was;
}

void prof_resume(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on;
}

void prof_read(int id, double* ms, int64_t* count) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  *ms = g_ms[id];
  *count = g_cnt[id];
}

const char* prof_name(int id) { return (id >= 0 && id < kProfKernels) ? kNames[id] : nullptr; }

}  // namespace ngs
