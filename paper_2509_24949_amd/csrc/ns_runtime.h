// Host-side pieces shared by the run API (ns_api.hip) and the serving
// scheduler (ns_server.hip): error reporting, device allocations of a run,
// the run object itself and its construction.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include "../../include/ns.h"
#include "ns_internal.h"

namespace ns {

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
  bool packed = false;               // launch configuration of the packed serving kernels
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
  }
};

namespace ns {
// Validate, allocate and fill a run: tables, initial population and its
// likelihoods, on stream st (synchronised before returning).  packed selects
// the launch configuration of the packed serving kernels (256 threads per
// chain, tables read through the caches), under which a run's arithmetic
// is the same alone and in any mix.
int run_create(ns_run** out, const ns_problem* P, const ns_opts* O, hipStream_t st, bool packed);
// Copy the device scalars into the pinned mirror (synchronises st).
int sync_state(ns_run* r);
}  // namespace ns
