// Internal interfaces between the host runtime (ns_api.hip) and the kernels
// (ns_kernels.hip) of libns.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ns_device.h"

namespace ns {

// Scalars of a run that live in device memory and are updated by kernels.
struct DevState {
  double logX, logZ, H, lstar;
  long long n_dead;
  long long n_evals;
  long long n_bin_terms;   // sum over evaluations of the active bins
  int iter;
  int done;        // 0 running, 1 criterion met, 2 dead-point capacity reached
  int walk_len;    // random-walk kernel: proposals per chain in the next iteration
  int pad;
};

// One iteration's metrics record as the termination kernel writes it; the
// layout is the public ns_iter_t's (checked where both are visible).
constexpr int PROBE_HIST = 32;
struct IterRec {
  int iter, probes_min, probes_max, pad;
  double lstar, logX, logZ, log_remaining;
  long long probes, steps, accepted, stepouts, shrinks;
  int hist[PROBE_HIST];
};

// Likelihood tables in HBM (built once per run).
struct Tables {
  const double* f;      // [n_bins] f_k
  const double* f13;    // [n_bins] f_k^(1/3)
  const double* lnf3;   // [n_bins] ln(f_k) / 3
  const double* fm53;   // [n_bins] f_k^(-5/3)
  const double2* dw;    // [n_det][n_bins] 4 df f_k^(-7/6) d_k / S_k
  const double* hpre;   // [n_det][n_bins] prefix sums of 4 df f^(-7/3) / S
  const float2* dw32;   // mixed form: dw * dw_scale in float (else null)
};

// Relative-binning tables: nb coarse bins whose nb+1 edges sit on grid
// frequencies; summary sums of the data against the fiducial waveform h0.
struct RBTables {
  int nb;
  const int* edge;        // [nb+1] fine-grid index of each edge
  const double* fe;       // [nb+1] edge frequency
  const double* fe13;     // [nb+1] fe^(1/3)
  const double* lnfe3;    // [nb+1] ln(fe) / 3
  const double* fem53;    // [nb+1] fe^(-5/3)
  const double* phi0;     // [n_det][nb+1] fiducial phase at the edges, detector delay included (cycles)
  const double2* g0;      // [n_det] 1 / (A0 K0_det) of the fiducial
  const double* fm;       // [nb] bin centres (fe_b + fe_{b+1}) / 2
  const double* inv_w;    // [nb] 1 / (fe_{b+1} - fe_b)
  const double2* A0;      // [n_det][nb] sum 4 df conj(d) h0 / S
  const double2* A1;      // [n_det][nb] sum 4 df conj(d) h0 / S (f - fm)
  const double* B0;       // [n_det][nb] sum 4 df |h0|^2 / S
  const double* B1;       // [n_det][nb] sum 4 df |h0|^2 / S (f - fm)
  // the same sums accumulated from each bin's first fine bin up to fine bin
  // k (inclusive), for the bin that straddles f_ISCO: [n_det][n_bins]
  const double2* cA0;
  const double2* cA1;
  const double* cB0;
  const double* cB1;
  // mixed form: the full-bin sums in float (else null)
  const float2* A0f;
  const float2* A1f;
  const float* B0f;
  const float* B1f;
  // the batched kernel's per-edge records (the linear model summed per edge)
  // and right-hand parts, [nb+1] each, layout fixed by the kernel
  const double* erec;
};

// Device buffers of one run.
struct RunDev {
  int n, k, d, m;
  double width;
  int max_stepout, max_shrink;
  double log_term;            // ln(term_frac), or -inf for "never"
  uint64_t key0, key1;
  long long cap;              // dead-point capacity
  DevState* state;
  double* u;                  // [n][d]
  double* lam;                // [n]
  int* rank;                  // [n]
  int* dead;                  // [k]
  int* surv;                  // [n] survivors of the iteration in ascending slot order (first n - k)
  int* start;                 // [k]
  double* chol;               // [d][d]
  int kernel;                 // 0 slice chains, 1 random-walk chains
  int walk_accept, walk_max;  // random walk: target acceptances per chain, chain-length cap
  int* acc;                   // [k] per chain in the last iteration: random walk, accepted
                              // proposals; slice, steps that moved
  int* probes;                // [k] likelihood calls of each chain in the last iteration
  long long* bins;            // [k] active bins summed over the chain's probes in the last iteration
  int* nso;                   // [k] slice: bracket expansions of each chain in the last iteration
  int* nsh;                   // [k] slice: rejected shrink candidates of each chain
  int move_counts;            // slice: the chains count their moves (nso, nsh, acc and the histogram)
  IterRec* trace;             // [trace_cap] per-iteration metrics
  int trace_cap;
  double* du;                 // [cap][d]
  double* dlam;               // [cap]
  double* dlogx;              // [cap]
  double* dlogw;              // [cap]
  int* diter;                 // [cap]
  int* dslot;                 // [cap]
  int* dnlive;                // [cap]
};

// Likelihood kernels: full grid and relative binning, each in double
// precision or in the mixed form (float sincos, products and bin sums;
// double phase), and the Gaussian test likelihood.
enum LikeKind { LK_FULL = 0, LK_RB = 1, LK_GAUSS = 2, LK_FULL32 = 3, LK_RB32 = 4 };
__host__ __device__ constexpr bool lk_full(int lk) { return lk == LK_FULL || lk == LK_FULL32; }
__host__ __device__ constexpr bool lk_rb(int lk) { return lk == LK_RB || lk == LK_RB32; }
__host__ __device__ constexpr bool lk_mixed(int lk) { return lk == LK_FULL32 || lk == LK_RB32; }

// Launch configuration chosen at init.
struct LaunchCfg {
  int slice_threads;          // 64, 128 or 256 threads per chain
  bool lds_tables;            // stage the full-grid tables in LDS
  bool move_counts;           // the move-counting chain kernels (64 threads per chain)
  size_t lds_bytes;           // dynamic LDS of the chain kernel
};

// A resident run as the packed (serving) kernels see it.
struct PackedRun {
  const ModelDev* M;
  Tables T;
  RBTables RB;
  RunDev R;
};

// ---- launch wrappers (ns_kernels.hip) --------------------------------------
// M is the host copy of the model, Md the same struct in device memory.
hipError_t launch_build_tables(const ModelDev& M, const ModelDev* Md, const double* data_re, const double* data_im,
                               const double* psd, double* f, double* f13, double* lnf3, double* fm53, double2* dw,
                               double* hpre, double* scratch, hipStream_t st);
// Log-likelihood of the data under the noise-only model into out[0]
// (device): sum over the n values of the Gaussian log-densities of the real
// and imaginary parts, each of variance psd / (4 df).
hipError_t launch_noise_loglike(const double* dre, const double* dim, const double* psd, long n, double df,
                                double* out, hipStream_t st);
hipError_t launch_init_live(const RunDev& R, hipStream_t st);
// Batched likelihood; terms (optional, device [n]) receives each probe's
// counted terms (full grid: active bins; relative binning: edges; Gaussian: 0).
// pbuf (optional, device [n]): probe coefficients, which select the two-pass
// full-grid form (set-up pass, then one wavefront per probe).
hipError_t launch_loglike(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                          const double* u, long n, double* out, int* terms, Probe* pbuf, hipStream_t st);
hipError_t launch_select(const double* lam, int n, int k, int* rank, int* dead, double* lstar, const int* done,
                         hipStream_t st);
// Device address of this device's probe-record scratch of ns_loglike_noalloc
// (NS_LOGLIKE_NOALLOC_MAX records, held by the library until the process
// ends).  The current device must be `device`; the address is looked up once
// per device (hipGetSymbolAddress) and cached.
hipError_t noalloc_probe_scratch(int device, Probe** out);
// Random-walk chains of one iteration (launch after the preparation kernel).
hipError_t launch_walk(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB, const RunDev& R,
                       hipStream_t st);
// ev (optional): five events recorded before select, after select, after
// prep, after the chains and after the termination kernel.
hipError_t launch_iteration(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                            const RunDev& R, const LaunchCfg& C, hipStream_t st, hipEvent_t* ev = nullptr);
hipError_t launch_waveform(const ModelDev& M, const ModelDev* Md, const double* theta_dev, int det, int apply_cut,
                           double* h_re, double* h_im, hipStream_t st);
hipError_t launch_final(const RunDev& R, int n_sim, double* out, hipStream_t st);
hipError_t launch_samples(const ModelDev* Md, const RunDev& R, long long total, double logZ, double* theta,
                          double* logl, double* logw, hipStream_t st);
// Systematic resampling into n_out equal-weight samples; cum: device
// [total + 1] scratch; idx: device [n_out]; theta: device [n_out][d] or NULL.
hipError_t launch_resample(const ModelDev* Md, const RunDev& R, long long total, double logZ, long long n_out,
                           double* cum, int* idx, double* theta, hipStream_t st);
// Relative-binning set-up: edges (edge_out receives a host copy for
// validation), fiducial phases and the summary sums.  w is the scratch array
// of per-bin weights 4 df f^(-7/3) / S written by launch_build_tables.
struct RBBuffers {
  int* edge; double *fe, *fe13, *lnfe3, *fem53, *phi0, *fm, *inv_w, *B0, *B1, *cB0, *cB1;
  double2 *g0, *A0, *A1, *cA0, *cA1;
  float2 *A0f, *A1f; float *B0f, *B1f;   // mixed form only
  double* erec;
};
// Doubles of the batched relative-binning kernel's edge records for nb coarse bins.
size_t rb_edge_record_doubles(int nb, int n_det, bool mixed);
hipError_t launch_build_rb_edge_records(const ModelDev& M, const RBTables& RB, double* erec, hipStream_t st);
// Mixed form: float copies of the data table (scaled) and of the bin sums.
hipError_t launch_to_float(const double2* src, float2* dst, size_t n, double scale, hipStream_t st);
hipError_t launch_to_float(const double* src, float* dst, size_t n, double scale, hipStream_t st);
hipError_t launch_build_rb_edges(const ModelDev* Md, int nb, const RBBuffers& B, hipStream_t st);
hipError_t launch_build_rb_sums(const ModelDev& M, const ModelDev* Md, const Tables& T, const double* hw,
                                const double* theta_fid_dev, int nb, const RBBuffers& B, hipStream_t st);
// Chain-kernel set-up of a run with n_chains chains: staged tables if they
// fit, then the widest workgroup (256, 128 or 64 threads) that keeps every
// chain resident at once; with count_moves, the move-counting kernels of 64
// threads per chain.
hipError_t configure_slice(const ModelDev& M, int rb_nb, int n_chains, bool count_moves, LaunchCfg* C);
// Chain-kernel set-up of runs that take part in packed launches: 64
// threads per chain (128 or 256 through NS_PACKED_THREADS, for tuning),
// tables read through the caches (as in the packed kernel).
hipError_t configure_slice_packed(const ModelDev& M, int rb_nb, LaunchCfg* C);
// One iteration of every run in `runs` (device array of nr descriptors):
// packed selection (rank_off: prefix of ceil(n_r/4) blocks), preparation,
// chain kernel (slice_off: prefix of k_r blocks) and termination.  lk is the
// shared likelihood kind (LK_FULL, LK_FULL32, LK_RB or LK_RB32), nt the shared
// threads per chain, slice_lds the largest chain-kernel LDS of the runs.
hipError_t launch_iteration_packed(const PackedRun* runs, const int* rank_off, const int* slice_off, int nr,
                                   int rank_blocks, int slice_blocks, int lk, int nt, size_t slice_lds,
                                   hipStream_t st);
// done flag of every run into out[nr].
hipError_t launch_gather_done(const PackedRun* runs, int nr, int* out, hipStream_t st);
int likelihood_kind(const ModelDev& M);

}  // namespace ns
