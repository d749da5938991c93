// Multi-grid groups: several plans (velocity grids, kernels, ranks) with their
// own item counts evaluated as one launch.  Each plan's pipeline runs on its
// own stream between a fork and a join event on the caller's stream, so grids
// of different sizes overlap on the GPU; the whole fork/join is captured once
// per pointer set into a hipGraph and replayed with a single hipGraphLaunch.
//
// Also here: the autotuner, which times the candidate schedules (fused or
// two-pass hot loop, items per chunk) of one plan on the caller's own inputs
// and keeps the fastest, optionally caching the choice in a text file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "qcoll_internal.h"

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

qcoll_status gfail(qcoll_status s, const std::string &m) {
  qcoll::set_error(m);
  return s;
}

// cost model used to order the branches: model work of one item
double item_cost(const qcoll::Plan &p) {
  const double n3 = double(p.n3());
  return double(p.N_rho) * p.M * n3 * std::log2(n3);
}

}  // namespace

struct qcoll_group_s {
  std::vector<qcoll_plan> plans;
  std::vector<int64_t> counts;
  std::vector<int> order;                  // plans by decreasing total cost
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr;
  int device = 0;
  struct Cached {
    std::vector<const void *> ptrs;
    std::vector<uint64_t> gens;   // plan generations at capture
    int32_t op = 0, flag = 0;
    void *ws = nullptr;
    hipStream_t st = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Cached> cache;
};

namespace {

size_t plan_bytes(const qcoll::Plan &p, int64_t count, int32_t op) {
  if (count <= 0) return 0;
  return al256(qcoll::make_layout(p, count, op).total);
}

// enqueue every branch of the group on its stream, fork/join on st
qcoll_status enqueue(qcoll_group g, int32_t op, const double *const *a, const double *const *b,
                     double *const *out, double *const *out2, int32_t flag, void *ws, hipStream_t st) {
  if (hipEventRecord(g->fork, st) != hipSuccess) return gfail(QCOLL_EDEVICE, "hipEventRecord failed");
  char *w = static_cast<char *>(ws);
  std::vector<size_t> off(g->plans.size());
  size_t o = 0;
  for (size_t i = 0; i < g->plans.size(); ++i) {
    off[i] = o;
    o += plan_bytes(g->plans[i]->p, g->counts[i], op);
  }
  for (int i : g->order) {
    const qcoll::Plan &p = g->plans[i]->p;
    const int64_t n = g->counts[i];
    if (n == 0) continue;
    hipStream_t s = g->streams[i];
    if (hipStreamWaitEvent(s, g->fork, 0) != hipSuccess) return gfail(QCOLL_EDEVICE, "hipStreamWaitEvent failed");
    const qcoll::Layout lay = qcoll::make_layout(p, n, op);
    qcoll_status rc;
    if (op == 0) {
      if ((rc = qcoll::launch_eval(p, n, a[i], out[i], w + off[i], lay, s)) != QCOLL_OK) return rc;
      if (flag && (rc = qcoll::launch_conserve(p, n, out[i], nullptr, s)) != QCOLL_OK) return rc;
    } else {
      if ((rc = qcoll::launch_vjp(p, n, a[i], b[i], out[i], out2 ? out2[i] : nullptr, flag != 0, w + off[i], lay,
                                  s)) != QCOLL_OK)
        return rc;
    }
    if (hipEventRecord(g->done[i], s) != hipSuccess) return gfail(QCOLL_EDEVICE, "hipEventRecord failed");
    if (hipStreamWaitEvent(st, g->done[i], 0) != hipSuccess) return gfail(QCOLL_EDEVICE, "hipStreamWaitEvent failed");
  }
  return QCOLL_OK;
}

qcoll_status run(qcoll_group g, int32_t op, const double *const *a, const double *const *b, double *const *out,
                 double *const *out2, int32_t flag, void *ws, size_t ws_bytes, void *stream, int32_t use_graph) {
  if (!g) return gfail(QCOLL_EINVAL, "group is NULL");
  const size_t need = qcoll_group_workspace_bytes(g, op);
  if (need && (!ws || ws_bytes < need)) return gfail(QCOLL_EWORKSPACE, "workspace missing or too small");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != g->device) return gfail(QCOLL_EINVAL, "wrong current device");
  for (size_t i = 0; i < g->plans.size(); ++i) {
    if (g->counts[i] == 0) continue;
    if (!a || !a[i] || !out || !out[i] || (op == 1 && (!b || !b[i])))
      return gfail(QCOLL_EINVAL, "NULL array for a plan with items");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!use_graph) return enqueue(g, op, a, b, out, out2, flag, ws, st);

  // a captured graph bakes in the plans' table pointers, schedules and
  // workspace layouts: the key holds every plan's generation besides the I/O
  // pointers, so a change to any plan (omega, schedule, chunk, autotune)
  // leads to a fresh capture
  std::vector<const void *> key;
  std::vector<uint64_t> gens;
  for (size_t i = 0; i < g->plans.size(); ++i) {
    key.push_back(a[i]);
    key.push_back(b ? b[i] : nullptr);
    key.push_back(out[i]);
    key.push_back(out2 ? out2[i] : nullptr);
    gens.push_back(g->plans[i]->p.gen);
  }
  for (auto &c : g->cache)
    if (c.ptrs == key && c.gens == gens && c.op == op && c.flag == flag && c.ws == ws && c.st == st) {
      if (hipGraphLaunch(c.exec, st) != hipSuccess) return gfail(QCOLL_EDEVICE, "hipGraphLaunch failed");
      return QCOLL_OK;
    }
  // capture once: kernels only (no memset nodes), timing events off
  const bool timing = qcoll::timing_on();
  qcoll_timing_enable(0);
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    qcoll_timing_enable(timing);
    return gfail(QCOLL_EDEVICE, "hipStreamBeginCapture failed (the default stream cannot be captured)");
  }
  qcoll_status rc = enqueue(g, op, a, b, out, out2, flag, ws, st);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(st, &graph);
  qcoll_timing_enable(timing);
  if (rc != QCOLL_OK) {
    if (graph) hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess || !graph) return gfail(QCOLL_EDEVICE, "hipStreamEndCapture failed");
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return gfail(QCOLL_EDEVICE, "hipGraphInstantiate failed");
  }
  (void)hipGraphDestroy(graph);
  if (g->cache.size() >= 8) {
    (void)hipGraphExecDestroy(g->cache.front().exec);
    g->cache.erase(g->cache.begin());
  }
  qcoll_group_s::Cached c;
  c.ptrs = key;
  c.gens = gens;
  c.op = op;
  c.flag = flag;
  c.ws = ws;
  c.st = st;
  c.exec = exec;
  g->cache.push_back(c);
  qcoll::log("group %p: captured graph %zu for op %d (%zu plans)", static_cast<void *>(g), g->cache.size(), op,
             g->plans.size());
  if (hipGraphLaunch(exec, st) != hipSuccess) return gfail(QCOLL_EDEVICE, "hipGraphLaunch failed");
  return QCOLL_OK;
}

}  // namespace

extern "C" {

qcoll_status qcoll_group_create(const qcoll_plan *plans, const int64_t *counts, int32_t nplans, qcoll_group *out) {
  if (!plans || !counts || !out || nplans < 1 || nplans > 64) return gfail(QCOLL_EINVAL, "need 1..64 plans");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return gfail(QCOLL_EDEVICE, "hipGetDevice failed");
  for (int i = 0; i < nplans; ++i) {
    if (!plans[i]) return gfail(QCOLL_EINVAL, "NULL plan");
    if (counts[i] < 0) return gfail(QCOLL_EINVAL, "negative item count");
    if (plans[i]->p.device != dev) return gfail(QCOLL_EINVAL, "plans must live on the current device");
  }
  auto *g = new (std::nothrow) qcoll_group_s;
  if (!g) return gfail(QCOLL_ENOMEM, "host allocation failed");
  g->device = dev;
  g->plans.assign(plans, plans + nplans);
  g->counts.assign(counts, counts + nplans);
  g->order.resize(nplans);
  for (int i = 0; i < nplans; ++i) g->order[i] = i;
  std::stable_sort(g->order.begin(), g->order.end(), [&](int x, int y) {
    return item_cost(g->plans[x]->p) * g->counts[x] > item_cost(g->plans[y]->p) * g->counts[y];
  });
  bool ok = hipEventCreateWithFlags(&g->fork, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < nplans && ok; ++i) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    g->streams.push_back(s);
    g->done.push_back(e);
  }
  if (!ok) {
    qcoll_group_destroy(g);
    return gfail(QCOLL_EDEVICE, "stream or event creation failed");
  }
  *out = g;
  return QCOLL_OK;
}

qcoll_status qcoll_group_destroy(qcoll_group g) {
  if (!g) return QCOLL_OK;
  for (auto &c : g->cache) hipGraphExecDestroy(c.exec);
  for (auto s : g->streams)
    if (s) hipStreamDestroy(s);
  for (auto e : g->done)
    if (e) hipEventDestroy(e);
  if (g->fork) hipEventDestroy(g->fork);
  delete g;
  return QCOLL_OK;
}

size_t qcoll_group_workspace_bytes(qcoll_group g, int32_t op) {
  if (!g || (op != 0 && op != 1)) return 0;
  size_t o = 0;
  for (size_t i = 0; i < g->plans.size(); ++i) o += plan_bytes(g->plans[i]->p, g->counts[i], op);
  return o;
}

qcoll_status qcoll_group_eval(qcoll_group g, const double *const *f, double *const *Q, int32_t conserve, void *ws,
                              size_t ws_bytes, void *stream, int32_t use_graph) {
  return run(g, 0, f, nullptr, Q, nullptr, conserve, ws, ws_bytes, stream, use_graph);
}

qcoll_status qcoll_group_vjp(qcoll_group g, const double *const *f, const double *const *gq, double *const *df,
                             double *const *domega, int32_t through_conserve, void *ws, size_t ws_bytes,
                             void *stream, int32_t use_graph) {
  if (g)
    for (size_t i = 0; i < g->plans.size(); ++i)
      if (g->plans[i]->p.literal || g->plans[i]->p.N > 48)
        return gfail(QCOLL_ENOTSUP, "the VJP needs plans with the symmetric Nyquist convention and N <= 48");
  if (g && domega)
    for (size_t i = 0; i < g->plans.size(); ++i)
      if (domega[i] && g->plans[i]->p.truncated)
        return gfail(QCOLL_ENOTSUP, "the omega gradient needs untruncated plans");
  if (!df) return gfail(QCOLL_EINVAL, "df is NULL");
  return run(g, 1, f, gq, df, domega, through_conserve, ws, ws_bytes, stream, use_graph);
}

// ---------------------------------------------------------------------------
// autotuner

qcoll_status qcoll_plan_set_chunk(qcoll_plan plan, int32_t items) {
  if (!plan) return gfail(QCOLL_EINVAL, "plan is NULL");
  if (items < 0 || items > 65536) return gfail(QCOLL_EINVAL, "chunk must be 0..65536");
  plan->p.chunk = items;
  ++plan->p.gen;
  qcoll::log("plan %p: chunk %d", static_cast<void *>(plan), items);
  return QCOLL_OK;
}

// candidate items per chunk of the autotuner: each nominal size c is
// balanced over the batch, ceil(batch / ceil(batch / c)), so that all
// launches of one eval have the same size; duplicates are dropped
static std::vector<int> tune_chunks(int64_t batch) {
  std::vector<int> out;
  for (int c : {32, 64, 96, 128, 192, 256}) {
    const int64_t n = (batch + c - 1) / c;
    const int ck = int((batch + n - 1) / n);
    if (std::find(out.begin(), out.end(), ck) == out.end()) out.push_back(ck);
  }
  return out;
}

size_t qcoll_autotune_workspace_bytes(qcoll_plan plan, int64_t batch) {
  if (!plan || batch <= 0) return 0;
  qcoll::Plan p = plan->p;  // copy: only schedule/chunk are varied
  size_t mx = 0;
  for (int sch : {1, 2})
    for (int ck : tune_chunks(batch)) {
      if (sch == 2 && !qcoll::onchip_schedule_supported(p)) continue;
      p.schedule = sch;
      p.chunk = ck;
      mx = std::max(mx, qcoll::make_layout(p, batch, 0).total);
    }
  return mx;
}

// Cache entries carry the schedule set they were timed against ("s2": the FP32
// fused kernels, the FP64 on-chip kernels at 16^3 and 32^3); a build that adds
// or changes a schedule bumps it, so that an older entry is timed again
// instead of pinning a plan to what used to be the faster schedule.
constexpr int kTuneScheduleSet = 2;

static std::string tune_key(const qcoll::Plan &p, int64_t batch) {
  int bucket = 1;
  while (bucket < batch && bucket < (1 << 20)) bucket <<= 1;
  std::ostringstream k;
  k << "gfx950 s" << kTuneScheduleSet << " N=" << p.N << " Nr=" << p.N_rho << " M=" << p.M
    << " prec=" << p.precision << " rank=" << p.rank << " batch<=" << bucket;
  return k.str();
}

qcoll_status qcoll_autotune(qcoll_plan plan, int64_t batch, const double *f, double *Q, void *ws, size_t ws_bytes,
                            void *stream, int32_t *host_schedule, int32_t *host_chunk) {
  if (!plan || batch <= 0 || !f || !Q) return gfail(QCOLL_EINVAL, "bad arguments");
  if (!ws || ws_bytes < qcoll_autotune_workspace_bytes(plan, batch))
    return gfail(QCOLL_EWORKSPACE, "workspace smaller than qcoll_autotune_workspace_bytes");
  qcoll::Plan &p = plan->p;
  const std::string key = tune_key(p, batch);
  const char *cache = std::getenv("QCOLL_AUTOTUNE_CACHE");
  if (cache) {
    std::ifstream in(cache);
    std::string line;
    while (std::getline(in, line)) {
      const size_t bar = line.find('|');
      if (bar == std::string::npos || line.substr(0, bar) != key) continue;
      // "<schedule> <chunk> [ms]": schedule 1 or 2, chunk 1..65536; anything
      // else (garbage, out-of-range numbers) is skipped
      const char *c0 = line.c_str() + bar + 1;
      char *e1 = nullptr, *e2 = nullptr;
      errno = 0;
      const long sch_l = std::strtol(c0, &e1, 10);
      const long ck_l = (e1 != c0) ? std::strtol(e1, &e2, 10) : 0;
      const bool parsed = errno == 0 && e1 != c0 && e2 && e2 != e1 && (sch_l == 1 || sch_l == 2) && ck_l >= 1 &&
                          ck_l <= 65536;
      const int sch = int(sch_l), ck = int(ck_l);
      if (parsed && (sch != 2 || qcoll::onchip_schedule_supported(p))) {
        p.schedule = sch;
        p.chunk = ck;
        ++p.gen;
        qcoll::log("autotune %s: cached schedule %d chunk %d (%s)", key.c_str(), sch, ck, cache);
        if (host_schedule) *host_schedule = sch;
        if (host_chunk) *host_chunk = ck;
        return QCOLL_OK;
      }
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return gfail(QCOLL_EDEVICE, "hipEventCreate failed");
  float best = 1e30f;
  int bs = p.schedule, bc = p.chunk;
  const bool timing = qcoll::timing_on();
  qcoll_timing_enable(0);
  qcoll_status rc = QCOLL_OK;
  for (int sch : {2, 1})
    for (int ck : tune_chunks(batch)) {
      if (sch == 2 && !qcoll::onchip_schedule_supported(p)) continue;
      p.schedule = sch;
      p.chunk = ck;
      const qcoll::Layout lay = qcoll::make_layout(p, batch, 0);
      if ((rc = qcoll::launch_eval(p, batch, f, Q, ws, lay, st)) != QCOLL_OK) break;  // warm-up
      // best of two timed runs
      float ms = 1e30f;
      for (int rep = 0; rep < 2 && rc == QCOLL_OK; ++rep) {
        if (hipEventRecord(e0, st) != hipSuccess) { rc = gfail(QCOLL_EDEVICE, "hipEventRecord failed"); break; }
        if ((rc = qcoll::launch_eval(p, batch, f, Q, ws, lay, st)) != QCOLL_OK) break;
        float t = 0.f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
          rc = gfail(QCOLL_EDEVICE, "autotune timing events failed");
          break;
        }
        ms = t < ms ? t : ms;
      }
      if (rc != QCOLL_OK) break;
      if (ms < best) {
        best = ms;
        bs = sch;
        bc = ck;
      }
    }
  qcoll_timing_enable(timing);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ++p.gen;   // the trial schedules changed the plan's layout
  if (rc != QCOLL_OK) return rc;
  p.schedule = bs;
  p.chunk = bc;
  qcoll::log("autotune %s: schedule %d chunk %d, %.3f ms", key.c_str(), bs, bc, best);
  if (host_schedule) *host_schedule = bs;
  if (host_chunk) *host_chunk = bc;
  if (cache) {
    std::ofstream outf(cache, std::ios::app);
    outf << key << "|" << bs << " " << bc << " " << best << "\n";
  }
  return QCOLL_OK;
}

size_t qcoll_group_autotune_workspace_bytes(qcoll_group g) {
  if (!g) return 0;
  size_t mx = 0;
  for (size_t i = 0; i < g->plans.size(); ++i)
    if (g->counts[i] > 0) mx = std::max(mx, qcoll_autotune_workspace_bytes(g->plans[i], g->counts[i]));
  return mx;
}

qcoll_status qcoll_group_autotune(qcoll_group g, const double *const *f, double *const *Q, void *ws, size_t ws_bytes,
                                  void *stream) {
  if (!g || !f || !Q) return gfail(QCOLL_EINVAL, "NULL argument");
  if (!ws || ws_bytes < qcoll_group_autotune_workspace_bytes(g))
    return gfail(QCOLL_EWORKSPACE, "workspace smaller than qcoll_group_autotune_workspace_bytes");
  for (size_t i = 0; i < g->plans.size(); ++i) {
    if (g->counts[i] == 0) continue;
    if (!f[i] || !Q[i]) return gfail(QCOLL_EINVAL, "NULL array for a plan with items");
    const qcoll_status rc = qcoll_autotune(g->plans[i], g->counts[i], f[i], Q[i], ws, ws_bytes, stream, nullptr,
                                           nullptr);
    if (rc != QCOLL_OK) return rc;
  }
  return QCOLL_OK;
}

}  // extern "C"
