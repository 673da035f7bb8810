// Status strings, version and the optional kernel timer.
#include <map>
#include <string>
#include <vector>

#include "famst_common.hpp"

namespace famst {

struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};

static bool g_prof = false;
static std::vector<ProfRec> g_recs;
static std::vector<hipEvent_t> g_pool;
static std::map<std::string, std::pair<int64_t, double>> g_acc;
static ProfRec g_open{nullptr, nullptr, nullptr};

static hipEvent_t pool_get() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

static void drain() {
  for (auto& r : g_recs) {
    float ms = 0.f;
    hipEventSynchronize(r.b);
    hipEventElapsedTime(&ms, r.a, r.b);
    auto& slot = g_acc[r.name];
    slot.first += 1;
    slot.second += ms;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
}

void prof_begin(const char* name, hipStream_t s) {
  if (!g_prof) return;
  g_open.name = name;
  g_open.a = pool_get();
  g_open.b = pool_get();
  hipEventRecord(g_open.a, s);
}

void prof_end(hipStream_t s) {
  if (!g_prof || !g_open.name) return;
  hipEventRecord(g_open.b, s);
  g_recs.push_back(g_open);
  g_open.name = nullptr;
  if (g_recs.size() > 4096) drain();
}

}  // namespace famst

using namespace famst;

extern "C" const char* famst_strerror(int status) {
  switch (status) {
    case FAMST_OK: return "ok";
    case FAMST_EINVAL: return "invalid argument";
    case FAMST_ECAPACITY: return "output capacity too small";
    case FAMST_EDISCONNECTED: return "edges do not span every cloud";
    case FAMST_EHIP: return "HIP runtime error";
    case FAMST_ENOTIMPL: return "combination not supported";
    case FAMST_ENONFINITE: return "input holds a NaN or an infinity";
    case FAMST_EWORKSPACE: return "workspace too small or misaligned";
    case FAMST_ETIMEOUT: return "a bounded wait inside a kernel ran out";
    case FAMST_WNOTCONVERGED: return "refinement stopped at max_rounds with edges still changing";
    default: return "unknown status";
  }
}

extern "C" int famst_version(void) { return 100; }

extern "C" int famst_profile_enable(int enable) {
  g_prof = enable != 0;
  return FAMST_OK;
}

extern "C" int famst_profile_reset(void) {
  drain();
  g_acc.clear();
  return FAMST_OK;
}

extern "C" int famst_profile_read(const char* name, int64_t* launches, double* total_ms) {
  if (!name || !launches || !total_ms) return FAMST_EINVAL;
  drain();
  auto it = g_acc.find(name);
  if (it == g_acc.end()) {
    *launches = 0;
    *total_ms = 0.0;
  } else {
    *launches = it->second.first;
    *total_ms = it->second.second;
  }
  return FAMST_OK;
}
