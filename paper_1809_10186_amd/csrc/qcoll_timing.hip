// Process-wide kernel timer: hipEvent pairs on the launch stream, per role name.
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "qcoll_internal.h"

namespace qcoll {
namespace {

struct Rec {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t open = 0;  // index of the pair awaiting its stop event
};

bool g_on = false;
std::string g_only;                 // empty: every role is timed
std::map<std::string, Rec> g_recs;
std::vector<hipEvent_t> g_pool;     // events of earlier rounds, reused (no create on the launch path)

hipEvent_t take_event() {
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

bool timing_on() { return g_on; }

void timing_begin(const char *name, hipStream_t st) {
  if (!g_only.empty() && g_only != name) return;
  Rec &r = g_recs[name];
  hipEvent_t a = take_event(), b = take_event();
  if (!a || !b) {
    if (a) g_pool.push_back(a);
    if (b) g_pool.push_back(b);
    return;
  }
  if (hipEventRecord(a, st) != hipSuccess) {
    g_pool.push_back(a);
    g_pool.push_back(b);
    return;
  }
  r.ev.emplace_back(a, b);
  r.open = r.ev.size();
}

void timing_end(const char *name, hipStream_t st) {
  auto it = g_recs.find(name);
  if (it == g_recs.end() || it->second.open == 0) return;
  (void)hipEventRecord(it->second.ev[it->second.open - 1].second, st);
  it->second.open = 0;
}

}  // namespace qcoll

extern "C" {

qcoll_status qcoll_timing_enable(int32_t on) {
  qcoll::g_on = on != 0;
  return QCOLL_OK;
}

qcoll_status qcoll_timing_select(const char *name) {
  qcoll::g_only = name ? name : "";
  return QCOLL_OK;
}

qcoll_status qcoll_timing_reset(void) {
  for (auto &kv : qcoll::g_recs)
    for (auto &e : kv.second.ev) {
      (void)hipEventSynchronize(e.second);
      qcoll::g_pool.push_back(e.first);
      qcoll::g_pool.push_back(e.second);
    }
  qcoll::g_recs.clear();
  return QCOLL_OK;
}

qcoll_status qcoll_timing_read(const char *name, double *ms, int64_t *count) {
  if (!name || !ms || !count) {
    qcoll::set_error("NULL argument");
    return QCOLL_EINVAL;
  }
  *ms = 0.0;
  *count = 0;
  auto it = qcoll::g_recs.find(name);
  if (it == qcoll::g_recs.end()) return QCOLL_OK;
  double tot = 0.0;
  int64_t n = 0;
  for (auto &e : it->second.ev) {
    if (hipEventSynchronize(e.second) != hipSuccess) {
      qcoll::set_error("hipEventSynchronize failed");
      return QCOLL_EDEVICE;
    }
    float t = 0.f;
    if (hipEventElapsedTime(&t, e.first, e.second) != hipSuccess) {
      qcoll::set_error("hipEventElapsedTime failed");
      return QCOLL_EDEVICE;
    }
    tot += t;
    ++n;
  }
  *ms = tot;
  *count = n;
  return QCOLL_OK;
}

qcoll_status qcoll_timing_names(char *buf, size_t cap) {
  if (!buf || cap == 0) {
    qcoll::set_error("NULL argument");
    return QCOLL_EINVAL;
  }
  std::string s;
  for (auto &kv : qcoll::g_recs) {
    if (!s.empty()) s += '\n';
    s += kv.first;
  }
  size_t n = s.size() < cap - 1 ? s.size() : cap - 1;
  s.copy(buf, n);
  buf[n] = '\0';
  return QCOLL_OK;
}

}  // extern "C"
