// Serving scheduler: a queue of sampling requests (one per event), admission
// of runs by device-memory footprint and slot count, and ticks that advance
// the resident runs by packed launches.  One launch per kernel covers the
// chains of all resident runs of a lane that share a likelihood form, so
// small runs fill the device together instead of one after another.
//
// Runs are sorted into lanes by the cost of one probe (detectors times the
// most bins a probe can have active): a packed chain launch lasts as long as
// its slowest chain, so a cheap run packed with a costly one would wait for
// it every iteration.  Each lane has its own stream, descriptor arrays and
// captured tick, and ticks on its own: a tick launches every idle lane and
// returns once some lane's tick has finished, so cheap runs advance many
// iterations while a costly lane works through one, and the lanes' launches
// overlap on the device.  Runs are built on a further stream, so admission
// does not wait for the lanes.
//
// Every resident run is built with the packed launch configuration (64
// threads per chain, tables read through the caches) and each workgroup of a
// packed launch computes exactly what the same workgroup computes when the run
// is alone, so a run's results do not depend on what else is resident.
#include <math.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <memory>
#include <thread>

#include "ns_runtime.h"

using namespace ns;

namespace {

constexpr int kMaxBypass = 16;   // admissions that may overtake the queue head
constexpr int kLanes = 3;
// lane boundaries in bin terms per probe (detectors x the most active bins)
constexpr long long kLaneCost[kLanes - 1] = {1024, 4096};

int lk_of(const ModelDev& M) {
  if (M.likelihood == NS_LIKE_RB) return M.mixed ? LK_RB32 : LK_RB;
  return M.mixed ? LK_FULL32 : LK_FULL;
}

int lane_of(const ModelDev& M) {
  const long long cost = (long long)M.n_det * M.k_lim;
  int l = 0;
  while (l < kLanes - 1 && cost >= kLaneCost[l]) ++l;
  return l;
}

// A submitted request with private copies of every host array it references.
struct Request {
  long long ticket = 0;
  ProblemCopy prob;
  ns_opts O{};
  size_t resident = 0, transient = 0;
  double t_submit = 0.0;
  int bypassed = 0;
};

struct Resident {
  long long ticket;
  ns_run* run;
  size_t bytes;
  double t_submit, t_admit;
  int lk;        // likelihood kind and threads per chain: runs that share
  int nt;        // both share a packed launch
};

struct Finished {
  ns_ticket_info info;
  ns_run* run;   // null after take, or when construction failed
  bool reported;
};

struct Group {
  int first, count, lk, nt, rank_blocks, slice_blocks;
  size_t lds;
};

// One cost class of resident runs with its own stream and packed-launch
// descriptors.  While a tick is in flight (busy) the descriptors and the
// first n_launched entries of running belong to the device; runs admitted in
// the meantime wait at the end of running for the next tick.
struct Lane {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  std::vector<Resident> running;
  PackedRun* d_runs = nullptr;
  int* d_off = nullptr;     // [2][max_runs]: chain-kernel then selection block offsets
  int* d_done = nullptr;    // [max_runs]
  PackedRun* h_runs = nullptr;
  int* h_off = nullptr;
  int* h_done = nullptr;
  std::vector<Group> groups;
  bool dirty = true;
  bool busy = false;
  int n_launched = 0;
  hipGraphExec_t exec = nullptr;
  int exec_iters = 0;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    exec_iters = 0;
  }
};

}  // namespace

struct ns_server {
  hipStream_t user_st = nullptr;   // runs taken from the server are handed over on it
  hipStream_t adm_st = nullptr;    // construction of admitted runs
  size_t budget = 0;
  int max_runs = 0;
  bool graph = false;
  size_t used = 0;   // resident and finished-but-not-taken runs
  long long next_ticket = 1;
  std::chrono::steady_clock::time_point t0;
  std::deque<std::unique_ptr<Request>> queue;
  Lane lanes[kLanes];
  std::vector<Finished> finished;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  int resident() const {
    int c = 0;
    for (const Lane& l : lanes) c += (int)l.running.size();
    return c;
  }
  ~ns_server() {
    for (Lane& l : lanes)
      if (l.st) (void)hipStreamSynchronize(l.st);
    if (adm_st) (void)hipStreamSynchronize(adm_st);
    for (Lane& l : lanes) {
      l.drop_graph();
      for (auto& r : l.running) delete r.run;
      if (l.d_runs) (void)hipFree(l.d_runs);
      if (l.d_off) (void)hipFree(l.d_off);
      if (l.d_done) (void)hipFree(l.d_done);
      if (l.h_runs) (void)hipHostFree(l.h_runs);
      if (l.h_off) (void)hipHostFree(l.h_off);
      if (l.h_done) (void)hipHostFree(l.h_done);
      if (l.ev) (void)hipEventDestroy(l.ev);
    }
    for (auto& f : finished) delete f.run;
    for (Lane& l : lanes)
      if (l.st) (void)hipStreamDestroy(l.st);
    if (adm_st) (void)hipStreamDestroy(adm_st);
  }
};

namespace {

// Admit queued requests in arrival order while slots and memory allow; a
// request that does not fit may be overtaken by later ones that do, until it
// has been overtaken kMaxBypass times.  Runs are built on the admission
// stream and join their lane's next tick.
int admit(ns_server* s) {
  bool head_blocked = false;
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    if (s->resident() >= s->max_runs) break;
    Request& q = **it;
    const bool fits = s->used + q.resident + q.transient <= s->budget;
    if (!fits) {
      if (it == s->queue.begin()) head_blocked = true;
      if (head_blocked && s->queue.front()->bypassed >= kMaxBypass) break;
      ++it;
      continue;
    }
    if (head_blocked) s->queue.front()->bypassed += 1;
    ns_run* r = nullptr;
    const double ta = s->now();
    const int rc = run_create(&r, &q.prob.P, &q.O, s->adm_st, true);
    if (rc != NS_OK) {
      Finished f{};
      f.info.ticket = q.ticket;
      f.info.status = rc;
      f.info.t_submit = q.t_submit;
      f.info.t_admit = ta;
      f.info.t_finish = s->now();
      f.run = nullptr;
      f.reported = false;
      s->finished.push_back(f);
    } else {
      Lane& l = s->lanes[lane_of(r->M)];
      r->st = l.st;      // built and synchronised on the admission stream; advanced on its lane's
      l.running.push_back(Resident{q.ticket, r, q.resident, q.t_submit, ta, lk_of(r->M), r->C.slice_threads});
      l.dirty = true;
      s->used += q.resident;
    }
    it = s->queue.erase(it);
  }
  return NS_OK;
}

// Group an idle lane's runs by likelihood form and chain-workgroup size and
// upload the descriptors.
int rebuild(ns_server* s, Lane& L) {
  L.drop_graph();
  std::stable_sort(L.running.begin(), L.running.end(), [](const Resident& a, const Resident& b) {
    return a.lk != b.lk ? a.lk < b.lk : a.nt < b.nt;
  });
  L.groups.clear();
  const int nr = (int)L.running.size();
  int* slice_off = L.h_off;
  int* rank_off = L.h_off + s->max_runs;
  for (int i = 0; i < nr; ++i) {
    const ns_run* r = L.running[i].run;
    L.h_runs[i] = PackedRun{r->Md, r->T, r->RB, r->R};
    if (L.groups.empty() || L.groups.back().lk != L.running[i].lk || L.groups.back().nt != L.running[i].nt)
      L.groups.push_back(Group{i, 0, L.running[i].lk, L.running[i].nt, 0, 0, 0});
    Group& g = L.groups.back();
    slice_off[i] = g.slice_blocks;
    rank_off[i] = g.rank_blocks;
    g.count += 1;
    g.slice_blocks += r->R.k;
    g.rank_blocks += (r->R.n + 3) / 4;
    g.lds = std::max(g.lds, r->C.lds_bytes);
  }
  if (nr > 0) {
    HIP_OK(hipMemcpyAsync(L.d_runs, L.h_runs, nr * sizeof(PackedRun), hipMemcpyHostToDevice, L.st));
    HIP_OK(hipMemcpyAsync(L.d_off, L.h_off, 2 * s->max_runs * sizeof(int), hipMemcpyHostToDevice, L.st));
  }
  L.dirty = false;
  return NS_OK;
}

hipError_t enqueue_iterations(ns_server* s, Lane& L, int n_iters) {
  for (int it = 0; it < n_iters; ++it)
    for (const Group& g : L.groups) {
      hipError_t e = launch_iteration_packed(L.d_runs + g.first, L.d_off + s->max_runs + g.first,
                                             L.d_off + g.first, g.count, g.rank_blocks, g.slice_blocks, g.lk,
                                             g.nt, g.lds, L.st);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

int launch_tick(ns_server* s, Lane& L, int n_iters) {
  if (!s->graph) {
    HIP_OK(enqueue_iterations(s, L, n_iters));
    return NS_OK;
  }
  if (!L.exec || L.exec_iters != n_iters) {
    L.drop_graph();
    hipGraph_t g = nullptr;
    HIP_OK(hipStreamBeginCapture(L.st, hipStreamCaptureModeRelaxed));
    const hipError_t e = enqueue_iterations(s, L, n_iters);
    const hipError_t e2 = hipStreamEndCapture(L.st, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(NS_E_HIP, "capturing a tick: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    const hipError_t e3 = hipGraphInstantiate(&L.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
      L.exec = nullptr;
      return fail(NS_E_HIP, "instantiating a tick: %s", hipGetErrorString(e3));
    }
    L.exec_iters = n_iters;
  }
  HIP_OK(hipGraphLaunch(L.exec, L.st));
  return NS_OK;
}

// Start a tick on an idle lane with resident runs: n_iters iterations of
// every run, then the runs' termination flags to the host and the lane's
// event.
int start_lane(ns_server* s, Lane& L, int n_iters) {
  int rc;
  if (L.dirty && (rc = rebuild(s, L))) return rc;
  const int nr = (int)L.running.size();
  if ((rc = launch_tick(s, L, n_iters))) return rc;
  HIP_OK(launch_gather_done(L.d_runs, nr, L.d_done, L.st));
  HIP_OK(hipMemcpyAsync(L.h_done, L.d_done, nr * sizeof(int), hipMemcpyDeviceToHost, L.st));
  HIP_OK(hipEventRecord(L.ev, L.st));
  L.n_launched = nr;
  L.busy = true;
  return NS_OK;
}

// A lane's tick has finished: retire the runs that terminated.
int finish_lane(ns_server* s, Lane& L) {
  const double tf = s->now();
  std::vector<Resident> keep;
  keep.reserve(L.running.size());
  for (int i = 0; i < (int)L.running.size(); ++i) {
    Resident& r = L.running[i];
    if (i >= L.n_launched || !L.h_done[i]) {
      keep.push_back(r);
      continue;
    }
    int rc;
    if ((rc = sync_state(r.run))) return rc;
    r.run->st = s->user_st;
    Finished f{};
    f.info.ticket = r.ticket;
    f.info.status = NS_OK;
    f.info.done = L.h_done[i];
    f.info.iterations = r.run->h_state->iter;
    f.info.t_submit = r.t_submit;
    f.info.t_admit = r.t_admit;
    f.info.t_finish = tf;
    f.info.bytes = r.bytes;
    f.run = r.run;
    f.reported = false;
    s->finished.push_back(f);
    L.dirty = true;
  }
  L.running.swap(keep);
  L.busy = false;
  return NS_OK;
}

}  // namespace

extern "C" {

int ns_server_create(ns_server** out, size_t hbm_budget, int max_runs, int flags, void* stream) {
  if (!out) return fail(NS_E_ARG, "out is NULL");
  *out = nullptr;
  if (max_runs < 1 || max_runs > 4096) return fail(NS_E_ARG, "max_runs must be in [1, 4096]");
  if (flags & ~NS_SERVER_GRAPH) return fail(NS_E_ARG, "unknown flags 0x%x", flags);
  if ((flags & NS_SERVER_GRAPH) && !stream) return fail(NS_E_ARG, "NS_SERVER_GRAPH needs a stream other than the null stream");
  std::unique_ptr<ns_server> s(new (std::nothrow) ns_server());
  if (!s) return fail(NS_E_OOM, "host allocation failed");
  s->user_st = static_cast<hipStream_t>(stream);
  s->max_runs = max_runs;
  s->graph = (flags & NS_SERVER_GRAPH) != 0;
  s->t0 = std::chrono::steady_clock::now();
  if (hbm_budget == 0) {
    size_t free_b = 0, total_b = 0;
    HIP_OK(hipMemGetInfo(&free_b, &total_b));
    hbm_budget = free_b / 10 * 9;
  }
  s->budget = hbm_budget;
  // the lanes' and the admission stream, at the default priority
  HIP_OK(hipStreamCreateWithFlags(&s->adm_st, hipStreamNonBlocking));
  for (Lane& l : s->lanes) {
    HIP_OK(hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&l.ev, hipEventDisableTiming));
    if (hipMalloc((void**)&l.d_runs, max_runs * sizeof(PackedRun)) != hipSuccess ||
        hipMalloc((void**)&l.d_off, 2 * max_runs * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&l.d_done, max_runs * sizeof(int)) != hipSuccess ||
        hipHostMalloc((void**)&l.h_runs, max_runs * sizeof(PackedRun), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&l.h_off, 2 * max_runs * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&l.h_done, max_runs * sizeof(int), hipHostMallocDefault) != hipSuccess)
      return fail(NS_E_OOM, "allocating the server's descriptor arrays failed");
    memset(l.h_off, 0, 2 * max_runs * sizeof(int));
  }
  *out = s.release();
  return NS_OK;
}

int ns_server_submit(ns_server* s, const ns_problem* P, const ns_opts* O, long long* ticket) {
  if (!s) return fail(NS_E_ARG, "server is NULL");
  ModelDev M;
  int rc = validate_and_model(P, &M);
  if (rc) return rc;
  if ((rc = validate_opts(O))) return rc;
  if (P->likelihood == NS_LIKE_GAUSS) return fail(NS_E_ARG, "the server takes the waveform likelihoods (FULL or RB)");
  if (O->kernel != NS_KERNEL_SLICE) return fail(NS_E_ARG, "the server runs slice-sampling chains only");
  std::unique_ptr<Request> q(new (std::nothrow) Request());
  if (!q) return fail(NS_E_OOM, "host allocation failed");
  run_footprint(P, O, &q->resident, &q->transient);
  if (q->resident + q->transient > s->budget)
    return fail(NS_E_OOM, "the run needs %zu device bytes, the server's budget is %zu", q->resident + q->transient,
                s->budget);
  q->prob.own(*P);
  q->O = *O;
  q->ticket = s->next_ticket++;
  q->t_submit = s->now();
  if (ticket) *ticket = q->ticket;
  s->queue.push_back(std::move(q));
  return NS_OK;
}

int ns_server_tick(ns_server* s, int n_iters, int* n_running, int* n_queued, int* n_finished) {
  TraceRange range_("ns_server_tick");
  if (!s) return fail(NS_E_ARG, "server is NULL");
  if (n_iters < 1 || n_iters > 1000) return fail(NS_E_ARG, "n_iters must be in [1, 1000]");
  int rc = admit(s);
  if (rc) return rc;
  for (Lane& l : s->lanes)
    if (!l.busy && !l.running.empty() && (rc = start_lane(s, l, n_iters))) return rc;
  // wait until some lane's tick has finished
  for (;;) {
    bool any_busy = false, finished_one = false;
    for (Lane& l : s->lanes) {
      if (!l.busy) continue;
      any_busy = true;
      const hipError_t e = hipEventQuery(l.ev);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return fail(NS_E_HIP, "a lane's tick: %s", hipGetErrorString(e));
      if ((rc = finish_lane(s, l))) return rc;
      finished_one = true;
    }
    if (finished_one || !any_busy) break;
    std::this_thread::yield();
  }
  if ((rc = admit(s))) return rc;
  // keep the device busy: idle lanes start their next tick before the caller
  // takes its results
  for (Lane& l : s->lanes)
    if (!l.busy && !l.running.empty() && (rc = start_lane(s, l, n_iters))) return rc;
  if (n_running) *n_running = s->resident();
  if (n_queued) *n_queued = (int)s->queue.size();
  if (n_finished) {
    int c = 0;
    for (const auto& f : s->finished) c += f.reported ? 0 : 1;
    *n_finished = c;
  }
  return NS_OK;
}

int ns_server_poll(ns_server* s, ns_ticket_info* out, int cap, int* n_out) {
  if (!s || (cap > 0 && !out) || cap < 0) return fail(NS_E_ARG, "bad poll arguments");
  int c = 0;
  for (auto& f : s->finished) {
    if (f.reported) continue;
    if (c >= cap) break;
    out[c++] = f.info;
    f.reported = true;
  }
  if (n_out) *n_out = c;
  return NS_OK;
}

int ns_server_take(ns_server* s, long long ticket, ns_run** out) {
  if (!s || !out) return fail(NS_E_ARG, "NULL argument");
  *out = nullptr;
  for (size_t i = 0; i < s->finished.size(); ++i) {
    Finished& f = s->finished[i];
    if (f.info.ticket != ticket) continue;
    if (!f.run) {
      const int status = f.info.status;
      s->finished.erase(s->finished.begin() + i);
      return fail(NS_E_STATE, "ticket %lld has no run (its construction failed with status %d)", ticket, status);
    }
    *out = f.run;
    s->used -= f.info.bytes;
    s->finished.erase(s->finished.begin() + i);
    return NS_OK;
  }
  for (const Lane& l : s->lanes)
    for (const auto& r : l.running)
      if (r.ticket == ticket) return fail(NS_E_STATE, "ticket %lld is still running", ticket);
  for (const auto& q : s->queue)
    if (q->ticket == ticket) return fail(NS_E_STATE, "ticket %lld is still queued", ticket);
  return fail(NS_E_ARG, "unknown or already taken ticket %lld", ticket);
}

int ns_server_info(ns_server* s, size_t* budget, size_t* used, int* n_running, int* n_queued) {
  if (!s) return fail(NS_E_ARG, "server is NULL");
  if (budget) *budget = s->budget;
  if (used) *used = s->used;
  if (n_running) *n_running = s->resident();
  if (n_queued) *n_queued = (int)s->queue.size();
  return NS_OK;
}

void ns_server_free(ns_server* s) { delete s; }

}  // extern "C"
