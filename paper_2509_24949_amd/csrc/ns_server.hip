// Serving scheduler: a queue of sampling requests (one per event), admission
// of runs by device-memory footprint and slot count, and ticks that advance
// every resident run by packed launches.  One launch per kernel covers the
// chains of all resident runs that share a likelihood form, so small runs
// fill the device together instead of one after another.
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

#include "ns_runtime.h"

using namespace ns;

namespace {

constexpr int kMaxBypass = 16;   // admissions that may overtake the queue head

int lk_of(const ModelDev& M) {
  if (M.likelihood == NS_LIKE_RB) return M.mixed ? LK_RB32 : LK_RB;
  return M.mixed ? LK_FULL32 : LK_FULL;
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

}  // namespace

struct ns_server {
  hipStream_t st = nullptr;
  size_t budget = 0;
  int max_runs = 0;
  bool graph = false;
  size_t used = 0;   // resident and finished-but-not-taken runs
  long long next_ticket = 1;
  std::chrono::steady_clock::time_point t0;
  std::deque<std::unique_ptr<Request>> queue;
  std::vector<Resident> running;
  std::vector<Finished> finished;
  // packed-launch descriptors: device arrays and their pinned host images
  PackedRun* d_runs = nullptr;
  int* d_off = nullptr;     // [2][max_runs]: chain-kernel then selection block offsets
  int* d_done = nullptr;    // [max_runs]
  PackedRun* h_runs = nullptr;
  int* h_off = nullptr;
  int* h_done = nullptr;
  std::vector<Group> groups;
  bool dirty = true;
  hipGraphExec_t exec = nullptr;
  int exec_iters = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    exec_iters = 0;
  }
  ~ns_server() {
    (void)hipStreamSynchronize(st);
    drop_graph();
    for (auto& r : running) delete r.run;
    for (auto& f : finished) delete f.run;
    if (d_runs) (void)hipFree(d_runs);
    if (d_off) (void)hipFree(d_off);
    if (d_done) (void)hipFree(d_done);
    if (h_runs) (void)hipHostFree(h_runs);
    if (h_off) (void)hipHostFree(h_off);
    if (h_done) (void)hipHostFree(h_done);
  }
};

namespace {

// Admit queued requests in arrival order while slots and memory allow; a
// request that does not fit may be overtaken by later ones that do, until it
// has been overtaken kMaxBypass times.
int admit(ns_server* s) {
  bool head_blocked = false;
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    if ((int)s->running.size() >= s->max_runs) break;
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
    const int rc = run_create(&r, &q.prob.P, &q.O, s->st, true);
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
      s->running.push_back(Resident{q.ticket, r, q.resident, q.t_submit, ta, lk_of(r->M), r->C.slice_threads});
      s->used += q.resident;
      s->dirty = true;
    }
    it = s->queue.erase(it);
  }
  return NS_OK;
}

// Group the resident runs by likelihood form and chain-workgroup size and
// upload the descriptors.
int rebuild(ns_server* s) {
  s->drop_graph();
  std::stable_sort(s->running.begin(), s->running.end(), [](const Resident& a, const Resident& b) {
    return a.lk != b.lk ? a.lk < b.lk : a.nt < b.nt;
  });
  s->groups.clear();
  const int nr = (int)s->running.size();
  int* slice_off = s->h_off;
  int* rank_off = s->h_off + s->max_runs;
  for (int i = 0; i < nr; ++i) {
    const ns_run* r = s->running[i].run;
    s->h_runs[i] = PackedRun{r->Md, r->T, r->RB, r->R};
    if (s->groups.empty() || s->groups.back().lk != s->running[i].lk || s->groups.back().nt != s->running[i].nt)
      s->groups.push_back(Group{i, 0, s->running[i].lk, s->running[i].nt, 0, 0, 0});
    Group& g = s->groups.back();
    slice_off[i] = g.slice_blocks;
    rank_off[i] = g.rank_blocks;
    g.count += 1;
    g.slice_blocks += r->R.k;
    g.rank_blocks += (r->R.n + 3) / 4;
    g.lds = std::max(g.lds, r->C.lds_bytes);
  }
  if (nr > 0) {
    HIP_OK(hipMemcpyAsync(s->d_runs, s->h_runs, nr * sizeof(PackedRun), hipMemcpyHostToDevice, s->st));
    HIP_OK(hipMemcpyAsync(s->d_off, s->h_off, 2 * s->max_runs * sizeof(int), hipMemcpyHostToDevice, s->st));
  }
  s->dirty = false;
  return NS_OK;
}

hipError_t enqueue_iterations(ns_server* s, int n_iters) {
  for (int it = 0; it < n_iters; ++it)
    for (const Group& g : s->groups) {
      hipError_t e = launch_iteration_packed(s->d_runs + g.first, s->d_off + s->max_runs + g.first,
                                             s->d_off + g.first, g.count, g.rank_blocks, g.slice_blocks, g.lk,
                                             g.nt, g.lds, s->st);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

int launch_tick(ns_server* s, int n_iters) {
  if (!s->graph) {
    HIP_OK(enqueue_iterations(s, n_iters));
    return NS_OK;
  }
  if (!s->exec || s->exec_iters != n_iters) {
    s->drop_graph();
    hipGraph_t g = nullptr;
    HIP_OK(hipStreamBeginCapture(s->st, hipStreamCaptureModeRelaxed));
    const hipError_t e = enqueue_iterations(s, n_iters);
    const hipError_t e2 = hipStreamEndCapture(s->st, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(NS_E_HIP, "capturing a tick: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    const hipError_t e3 = hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
      s->exec = nullptr;
      return fail(NS_E_HIP, "instantiating a tick: %s", hipGetErrorString(e3));
    }
    s->exec_iters = n_iters;
  }
  HIP_OK(hipGraphLaunch(s->exec, s->st));
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
  s->st = static_cast<hipStream_t>(stream);
  s->max_runs = max_runs;
  s->graph = (flags & NS_SERVER_GRAPH) != 0;
  s->t0 = std::chrono::steady_clock::now();
  if (hbm_budget == 0) {
    size_t free_b = 0, total_b = 0;
    HIP_OK(hipMemGetInfo(&free_b, &total_b));
    hbm_budget = free_b / 10 * 9;
  }
  s->budget = hbm_budget;
  if (hipMalloc((void**)&s->d_runs, max_runs * sizeof(PackedRun)) != hipSuccess ||
      hipMalloc((void**)&s->d_off, 2 * max_runs * sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&s->d_done, max_runs * sizeof(int)) != hipSuccess ||
      hipHostMalloc((void**)&s->h_runs, max_runs * sizeof(PackedRun), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&s->h_off, 2 * max_runs * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&s->h_done, max_runs * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return fail(NS_E_OOM, "allocating the server's descriptor arrays failed");
  memset(s->h_off, 0, 2 * max_runs * sizeof(int));
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
  if (!s) return fail(NS_E_ARG, "server is NULL");
  if (n_iters < 1 || n_iters > 1000) return fail(NS_E_ARG, "n_iters must be in [1, 1000]");
  int rc = admit(s);
  if (rc) return rc;
  if (s->dirty && (rc = rebuild(s))) return rc;
  const int nr = (int)s->running.size();
  if (nr > 0) {
    if ((rc = launch_tick(s, n_iters))) return rc;
    HIP_OK(launch_gather_done(s->d_runs, nr, s->d_done, s->st));
    HIP_OK(hipMemcpyAsync(s->h_done, s->d_done, nr * sizeof(int), hipMemcpyDeviceToHost, s->st));
    HIP_OK(hipStreamSynchronize(s->st));
    const double tf = s->now();
    std::vector<Resident> keep;
    keep.reserve(nr);
    for (int i = 0; i < nr; ++i) {
      Resident& r = s->running[i];
      if (!s->h_done[i]) {
        keep.push_back(r);
        continue;
      }
      if ((rc = sync_state(r.run))) return rc;
      Finished f{};
      f.info.ticket = r.ticket;
      f.info.status = NS_OK;
      f.info.done = s->h_done[i];
      f.info.iterations = r.run->h_state->iter;
      f.info.t_submit = r.t_submit;
      f.info.t_admit = r.t_admit;
      f.info.t_finish = tf;
      f.info.bytes = r.bytes;
      f.run = r.run;
      f.reported = false;
      s->finished.push_back(f);
      s->dirty = true;
    }
    s->running.swap(keep);
  }
  if ((rc = admit(s))) return rc;
  if (n_running) *n_running = (int)s->running.size();
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
  for (const auto& r : s->running)
    if (r.ticket == ticket) return fail(NS_E_STATE, "ticket %lld is still running", ticket);
  for (const auto& q : s->queue)
    if (q->ticket == ticket) return fail(NS_E_STATE, "ticket %lld is still queued", ticket);
  return fail(NS_E_ARG, "unknown or already taken ticket %lld", ticket);
}

int ns_server_info(ns_server* s, size_t* budget, size_t* used, int* n_running, int* n_queued) {
  if (!s) return fail(NS_E_ARG, "server is NULL");
  if (budget) *budget = s->budget;
  if (used) *used = s->used;
  if (n_running) *n_running = (int)s->running.size();
  if (n_queued) *n_queued = (int)s->queue.size();
  return NS_OK;
}

void ns_server_free(ns_server* s) { delete s; }

}  // extern "C"
