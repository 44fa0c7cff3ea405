// Host-side pieces shared by the run API (ns_api.hip) and the serving
// scheduler (ns_server.hip): error reporting, device allocations of a run,
// the run object itself and its construction.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/ns.h"
#include "ns_internal.h"

namespace ns {

// A named range on the calling thread for the profiler's marker trace
// (rocprofv3 --marker-trace): each public call of the library opens one for
// its duration.  Without a profiler attached the calls cost a few
// nanoseconds.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// Record a message for ns_last_error() and return code.
int fail(int code, const char* fmt, ...);

#define HIP_OK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return ::ns::fail(NS_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Device allocations of one run, released together.
struct DevMem {
  std::vector<void*> ptrs;
  ~DevMem() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  hipError_t alloc(T** out, size_t count) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(p);
    *out = static_cast<T*>(p);
    return e;
  }
};

// A problem with private copies of every host array it references.
struct ProblemCopy {
  ns_problem P{};
  std::vector<int> kind, per;
  std::vector<double> lo, hi, dre, dim, psd, geom, fid, mu;

  // p must have passed validation (array lengths follow from its sizes).
  void own(const ns_problem& p) {
    P = p;
    const size_t nd = p.n_dim;
    const size_t nbd = p.likelihood == NS_LIKE_GAUSS ? 0 : (size_t)p.n_det * p.n_bins;
    kind.assign(p.prior_kind, p.prior_kind + nd);
    lo.assign(p.prior_lo, p.prior_lo + nd);
    hi.assign(p.prior_hi, p.prior_hi + nd);
    P.prior_kind = kind.data();
    P.prior_lo = lo.data();
    P.prior_hi = hi.data();
    P.data_re = P.data_im = P.psd = P.det_geom = P.rb_fiducial = P.gauss_mu = nullptr;
    P.periodic = nullptr;
    per.clear();
    if (p.periodic) {
      per.assign(p.periodic, p.periodic + nd);
      P.periodic = per.data();
    }
    if (nbd) {
      dre.assign(p.data_re, p.data_re + nbd);
      dim.assign(p.data_im, p.data_im + nbd);
      psd.assign(p.psd, p.psd + nbd);
      P.data_re = dre.data();
      P.data_im = dim.data();
      P.psd = psd.data();
    }
    if (p.likelihood != NS_LIKE_GAUSS && p.model != NS_MODEL_TF2_4P && p.det_geom) {
      geom.assign(p.det_geom, p.det_geom + 9 * (size_t)p.n_det);
      P.det_geom = geom.data();
    }
    if (p.likelihood == NS_LIKE_RB && p.rb_fiducial) {
      fid.assign(p.rb_fiducial, p.rb_fiducial + nd);
      P.rb_fiducial = fid.data();
    }
    if (p.likelihood == NS_LIKE_GAUSS && p.gauss_mu) {
      mu.assign(p.gauss_mu, p.gauss_mu + nd);
      P.gauss_mu = mu.data();
    }
  }
};

int validate_and_model(const ns_problem* P, ModelDev* M);
int validate_opts(const ns_opts* o);

// Device bytes a run of (P, O) holds while resident, and the extra bytes its
// construction needs for a moment (staging of data and PSD), each allocation
// rounded up to 4 KiB.  P and O must have passed validation.
void run_footprint(const ns_problem* P, const ns_opts* O, size_t* resident, size_t* transient);

}  // namespace ns

struct ns_run {
  ns::ModelDev M{};
  ns::ModelDev* Md = nullptr;        // device copy of M
  ns::Tables T{};
  ns::RBTables RB{};
  ns::RunDev R{};
  ns::LaunchCfg C{};
  hipStream_t st = nullptr;
  int device = -1;                   // the device current at construction
  bool packed = false;               // launch configuration of the packed serving kernels
  ns::ProblemCopy prob;              // the problem as given (for ns_save)
  ns_opts opts{};
  double noise_loglike = 0.0;        // log-likelihood of the data under the noise-only model
  ns::Probe* probe_buf = nullptr;    // coefficients of a batched likelihood call (grown on demand)
  long probe_cap = 0;
  ns::DevMem mem;
  ns::DevState* h_state = nullptr;   // pinned mirror of the device scalars
  bool profiling = false;
  std::vector<std::array<hipEvent_t, 5>> events;   // per profiled iteration
  void release_events() {
    for (auto& a : events)
      for (hipEvent_t e : a) (void)hipEventDestroy(e);
    events.clear();
  }
  ~ns_run() {
    release_events();
    if (h_state) (void)hipHostFree(h_state);
    if (probe_buf) (void)hipFree(probe_buf);
  }
};

namespace ns {
// Validate, allocate and fill a run: tables, initial population and its
// likelihoods, on stream st (synchronised before returning).  packed selects
// the launch configuration of the packed serving kernels (64 threads per
// chain, tables read through the caches), under which a run's arithmetic
// is the same alone and in any mix.
int run_create(ns_run** out, const ns_problem* P, const ns_opts* O, hipStream_t st, bool packed);
// Copy the device scalars into the pinned mirror (synchronises st).
int sync_state(ns_run* r);
}  // namespace ns
