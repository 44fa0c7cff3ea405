// Host-side launchers of libns and the instantiations of every kernel other
// than the chain kernels (the device code is in ns_kernels.h).
#include <mutex>

#include "../../include/ns.h"
#include "ns_kernels.h"

namespace ns {

int likelihood_kind(const ModelDev& M) { return M.likelihood; }

hipError_t configure_slice(const ModelDev& M, int rb_nb, int n_chains, bool count_moves, LaunchCfg* C) {
  C->move_counts = count_moves;
  if (M.likelihood == LK_GAUSS) {
    C->slice_threads = 64;
    C->lds_tables = false;
    C->lds_bytes = slice_lds_fixed(64, count_moves);
    return hipSuccess;
  }
  const bool rb = M.likelihood == LK_RB;
  // LDS of a chain workgroup: its own data and the staged tables (optional)
  const size_t tab = rb ? rb_stage_doubles(rb_nb, M.n_det, M.mixed != 0) * sizeof(double)
                        : staged_table_bytes(M.k_lim, M.n_det, M.mixed != 0);
  auto lds_of = [&](int nt, bool stage) { return slice_lds_fixed(nt, count_moves) + (stage ? tab : 0); };
  // every chain should be resident at once: a CU holds eight waves of the
  // chain kernel (its registers allow two per SIMD) and 160 KB of LDS
  auto resident = [&](int nt, bool stage) {
    const long by_waves = 8 / (nt / 64);
    const long by_lds = (long)(160 * 1024 / lds_of(nt, stage));
    return 256L * (by_waves < by_lds ? by_waves : by_lds);
  };
  int force_nt = 0;
  if (const char* ev = getenv("NS_SLICE_THREADS")) {      // tuning override: 64, 128 or 256
    const int v = atoi(ev);
    if (v == 64 || v == 128 || v == 256) force_nt = v;
  }
  if (count_moves) force_nt = 64;                          // the move-counting kernels' width
  bool allow_stage = true;
  if (const char* ev = getenv("NS_LDS_TABLES")) allow_stage = atoi(ev) != 0;   // tuning override
  // prefer staged tables, then the widest workgroup that keeps every chain resident
  int nt = 64;
  bool stage = false, found = false;
  for (int pass = 0; pass < 2 && !found; ++pass) {
    const bool st = pass == 0;
    if (st && !allow_stage) continue;
    for (int cand = 256; cand >= 64 && !found; cand /= 2) {
      if (force_nt && cand != force_nt) continue;
      if (resident(cand, st) >= n_chains) { nt = cand; stage = st; found = true; }
    }
  }
  if (!found) {   // more chains than resident slots: the narrowest workgroup
    nt = force_nt ? force_nt : 64;
    stage = allow_stage && lds_of(nt, true) <= 80 * 1024;
  }
  C->slice_threads = nt;
  C->lds_tables = stage;
  C->lds_bytes = lds_of(nt, stage);
  return hipSuccess;
}

hipError_t launch_build_tables(const ModelDev& M, const ModelDev* Md, const double* dre, const double* dim,
                               const double* psd, double* f, double* f13, double* lnf3, double* fm53, double2* dw,
                               double* hpre, double* scratch, hipStream_t st) {
  const int nb = (M.n_bins + 255) / 256;
  hipLaunchKernelGGL(k_build_tables, dim3(nb), dim3(256), 0, st, Md, dre, dim, psd, f, f13, lnf3, fm53, dw,
                     scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prefix_rows, dim3(M.n_det), dim3(1024), 0, st, scratch, hpre, M.n_bins);
  return hipGetLastError();
}

hipError_t launch_noise_loglike(const double* dre, const double* dim, const double* psd, long n, double df,
                                double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_noise_loglike, dim3(1), dim3(1024), 0, st, dre, dim, psd, n, df, out);
  return hipGetLastError();
}

hipError_t launch_init_live(const RunDev& R, hipStream_t st) {
  hipLaunchKernelGGL(k_init_live, dim3((R.n + 255) / 256), dim3(256), 0, st, R.n, R.d, R.key0, R.key1, R.u);
  return hipGetLastError();
}

size_t rb_edge_record_doubles(int nb, int n_det, bool mixed) {
  return (size_t)(nb + 1) * (rb_lane_rec_doubles(n_det, mixed) + rb_lane_right_doubles(n_det, mixed));
}

hipError_t launch_build_rb_edge_records(const ModelDev& M, const RBTables& RB, double* erec, hipStream_t st) {
  const dim3 grid((unsigned)((RB.nb + 1 + 127) / 128)), block(128);
  const bool mx = M.mixed != 0;
  switch (M.n_det) {
    case 1: if (mx) hipLaunchKernelGGL((k_rb_edge_records<1, true>), grid, block, 0, st, RB, erec);
            else hipLaunchKernelGGL((k_rb_edge_records<1, false>), grid, block, 0, st, RB, erec);
            break;
    case 2: if (mx) hipLaunchKernelGGL((k_rb_edge_records<2, true>), grid, block, 0, st, RB, erec);
            else hipLaunchKernelGGL((k_rb_edge_records<2, false>), grid, block, 0, st, RB, erec);
            break;
    default: if (mx) hipLaunchKernelGGL((k_rb_edge_records<3, true>), grid, block, 0, st, RB, erec);
             else hipLaunchKernelGGL((k_rb_edge_records<3, false>), grid, block, 0, st, RB, erec);
             break;
  }
  return hipGetLastError();
}

// lanes per probe in the relative-binning batch (1 or 2)
constexpr int RB_LANE_HALVES = 2;

template <int NDET, bool MX>
hipError_t launch_loglike_rb_t(const ModelDev* Md, const RBTables& RB, int n_bins, const double* u, long n,
                               double* out, int* terms, Probe* pbuf, hipStream_t st) {
  (void)n_bins;
  (void)pbuf;
  if (n <= 0) return hipSuccess;
  // the edge records in LDS when they fit in 64 KB (up to about 300 coarse
  // bins), else read from the device array
  const size_t ne = (size_t)RB.nb + 1;
  const size_t lds = (ne * (rb_lane_rec_doubles(NDET, MX) + rb_lane_right_doubles(NDET, MX)) + (ne + 1) / 2) *
                     sizeof(double);
  constexpr int H = RB_LANE_HALVES;
  const size_t recs = H == 2 ? (256 / H) * sizeof(ProbeRec) : 0;   // the split set-up's records
  const dim3 grid((unsigned)((n + 256 / H - 1) / (256 / H)));
  if (lds <= 64 * 1024)
    hipLaunchKernelGGL((k_rb_lane<NDET, MX, true, H>), grid, dim3(256), lds + recs, st, Md, RB, u, n, out, terms);
  else
    hipLaunchKernelGGL((k_rb_lane<NDET, MX, false, H>), grid, dim3(256), recs, st, Md, RB, u, n, out, terms);
  return hipGetLastError();
}

// Probe records of ns_loglike_noalloc: every device holds its own copy of
// this array from the first use of the library until the process ends.  In
// host code its name is not a device address; kernels receive the address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) Probe scratch[NS_LOGLIKE_NOALLOC_MAX];

hipError_t noalloc_probe_scratch(int device, Probe** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static Probe* addr[kMaxDevices] = {};
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<Probe*>(p);
  }
  *out = addr[device];
  return hipSuccess;
}

hipError_t launch_loglike(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                          const double* u, long n, double* out, int* terms, Probe* pbuf, hipStream_t st) {
  if (M.likelihood == LK_GAUSS) return launch_loglike_t<1, LK_GAUSS, false>(M, Md, T, RB, u, n, out, terms, pbuf, st);
  if (M.likelihood == LK_RB) {
    if (M.mixed) {
      switch (M.n_det) {
        case 1: return launch_loglike_rb_t<1, true>(Md, RB, M.n_bins, u, n, out, terms, pbuf, st);
        case 2: return launch_loglike_rb_t<2, true>(Md, RB, M.n_bins, u, n, out, terms, pbuf, st);
        default: return launch_loglike_rb_t<3, true>(Md, RB, M.n_bins, u, n, out, terms, pbuf, st);
      }
    }
    switch (M.n_det) {
      case 1: return launch_loglike_rb_t<1, false>(Md, RB, M.n_bins, u, n, out, terms, pbuf, st);
      case 2: return launch_loglike_rb_t<2, false>(Md, RB, M.n_bins, u, n, out, terms, pbuf, st);
      default: return launch_loglike_rb_t<3, false>(Md, RB, M.n_bins, u, n, out, terms, pbuf, st);
    }
  }
  const bool lds = staged_table_bytes(M.k_lim, M.n_det, M.mixed != 0) <= 64 * 1024;
  if (M.mixed) {
    switch (M.n_det) {
      case 1: return lds ? launch_loglike_t<1, LK_FULL32, true>(M, Md, T, RB, u, n, out, terms, pbuf, st)
                         : launch_loglike_t<1, LK_FULL32, false>(M, Md, T, RB, u, n, out, terms, pbuf, st);
      case 2: return lds ? launch_loglike_t<2, LK_FULL32, true>(M, Md, T, RB, u, n, out, terms, pbuf, st)
                         : launch_loglike_t<2, LK_FULL32, false>(M, Md, T, RB, u, n, out, terms, pbuf, st);
      default: return lds ? launch_loglike_t<3, LK_FULL32, true>(M, Md, T, RB, u, n, out, terms, pbuf, st)
                          : launch_loglike_t<3, LK_FULL32, false>(M, Md, T, RB, u, n, out, terms, pbuf, st);
    }
  }
  switch (M.n_det) {
    case 1: return lds ? launch_loglike_t<1, LK_FULL, true>(M, Md, T, RB, u, n, out, terms, pbuf, st)
                       : launch_loglike_t<1, LK_FULL, false>(M, Md, T, RB, u, n, out, terms, pbuf, st);
    case 2: return lds ? launch_loglike_t<2, LK_FULL, true>(M, Md, T, RB, u, n, out, terms, pbuf, st)
                       : launch_loglike_t<2, LK_FULL, false>(M, Md, T, RB, u, n, out, terms, pbuf, st);
    default: return lds ? launch_loglike_t<3, LK_FULL, true>(M, Md, T, RB, u, n, out, terms, pbuf, st)
                        : launch_loglike_t<3, LK_FULL, false>(M, Md, T, RB, u, n, out, terms, pbuf, st);
  }
}

hipError_t launch_select(const double* lam, int n, int k, int* rank, int* dead, double* lstar, const int* done,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_rank, dim3((n + 3) / 4), dim3(256), 0, st, lam, n, k, rank, dead, lstar, done);
  return hipGetLastError();
}

hipError_t launch_iteration(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                            const RunDev& R, const LaunchCfg& C, hipStream_t st, hipEvent_t* ev) {
  hipError_t e;
  if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
  e = launch_select(R.lam, R.n, R.k, R.rank, R.dead, nullptr, &R.state->done, st);
  if (e != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_prep, dim3(1), dim3(1024), 0, st, R);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
  if (R.kernel == 1) {
    e = launch_walk(M, Md, T, RB, R, st);
  } else if (M.likelihood == LK_GAUSS) {
    e = C.move_counts ? launch_slice_t<1, 64, LK_GAUSS, false, true>(Md, T, RB, R, C.lds_bytes, st)
                      : launch_slice_t<1, 64, LK_GAUSS, false>(Md, T, RB, R, C.lds_bytes, st);
  } else if (C.move_counts) {
    switch (M.n_det) {
      case 1: e = launch_slice_mv_d1(M, Md, T, RB, R, C, st); break;
      case 2: e = launch_slice_mv_d2(M, Md, T, RB, R, C, st); break;
      default: e = launch_slice_mv_d3(M, Md, T, RB, R, C, st); break;
    }
  } else {
    switch (M.n_det) {
      case 1: e = launch_slice_d1(M, Md, T, RB, R, C, st); break;
      case 2: e = launch_slice_d2(M, Md, T, RB, R, C, st); break;
      default: e = launch_slice_d3(M, Md, T, RB, R, C, st); break;
    }
  }
  if (e != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[3], st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_term, dim3(1), dim3(1024), 0, st, R);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[4], st)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t configure_slice_packed(const ModelDev& M, int rb_nb, LaunchCfg* C) {
  // a resident mix already holds thousands of chains: one wave per chain
  // keeps the most chains in flight and wastes the fewest lanes on short probes
  C->slice_threads = 64;
  if (const char* ev = getenv("NS_PACKED_THREADS")) {     // tuning override: 64, 128 or 256
    const int v = atoi(ev);
    if (v == 64 || v == 128 || v == 256) C->slice_threads = v;
  }
  C->lds_tables = false;
  C->move_counts = false;
  C->lds_bytes = slice_lds_fixed(C->slice_threads, false);
  (void)rb_nb;
  return hipSuccess;
}


hipError_t launch_iteration_packed(const PackedRun* runs, const int* rank_off, const int* slice_off, int nr,
                                   int rank_blocks, int slice_blocks, int lk, int nt, size_t slice_lds,
                                   hipStream_t st) {
  if (nr <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rank_packed, dim3(rank_blocks), dim3(256), 0, st, runs, rank_off, nr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prep_packed, dim3(nr), dim3(1024), 0, st, runs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  switch (nt) {
    case 64: e = launch_slice_packed64(runs, slice_off, nr, slice_blocks, lk, slice_lds, st); break;
    case 128: e = launch_slice_packed128(runs, slice_off, nr, slice_blocks, lk, slice_lds, st); break;
    default: e = launch_slice_packed256(runs, slice_off, nr, slice_blocks, lk, slice_lds, st); break;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_term_packed, dim3(nr), dim3(1024), 0, st, runs);
  return hipGetLastError();
}

hipError_t launch_gather_done(const PackedRun* runs, int nr, int* out, hipStream_t st) {
  if (nr <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_done, dim3((nr + 255) / 256), dim3(256), 0, st, runs, nr, out);
  return hipGetLastError();
}

hipError_t launch_waveform(const ModelDev& M, const ModelDev* Md, const double* theta_dev, int det, int apply_cut,
                           double* h_re, double* h_im, hipStream_t st) {
  hipLaunchKernelGGL(k_waveform, dim3((M.n_bins + 255) / 256), dim3(256), 0, st, Md, theta_dev, det, apply_cut,
                     h_re, h_im);
  return hipGetLastError();
}

hipError_t launch_build_rb_edges(const ModelDev* Md, int nb, const RBBuffers& B, hipStream_t st) {
  hipLaunchKernelGGL(k_rb_edges, dim3((nb + 1 + 255) / 256), dim3(256), 0, st, Md, nb, B.edge, B.fe, B.fe13, B.lnfe3,
                     B.fem53);
  return hipGetLastError();
}

hipError_t launch_build_rb_sums(const ModelDev& M, const ModelDev* Md, const Tables& T, const double* hw,
                                const double* theta_fid_dev, int nb, const RBBuffers& B, hipStream_t st) {
  hipLaunchKernelGGL(k_rb_fiducial, dim3((nb + 1 + 255) / 256), dim3(256), 0, st, Md, theta_fid_dev, nb, B.fe, B.fe13,
                     B.lnfe3, B.fem53, B.phi0, B.g0, B.fm, B.inv_w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rb_sums, dim3((nb + 63) / 64, M.n_det), dim3(64), 0, st, Md, T, hw, theta_fid_dev, nb, B.edge,
                     B.fm, B.A0, B.A1, B.B0, B.B1, B.cA0, B.cA1, B.cB0, B.cB1);
  return hipGetLastError();
}

hipError_t launch_to_float(const double2* src, float2* dst, size_t n, double scale, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_float2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n, scale);
  return hipGetLastError();
}

hipError_t launch_to_float(const double* src, float* dst, size_t n, double scale, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_float1, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n, scale);
  return hipGetLastError();
}

hipError_t launch_final(const RunDev& R, int n_sim, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_final, dim3(1 + (n_sim > 0 ? n_sim : 0)), dim3(1024), 0, st, R, n_sim, out);
  return hipGetLastError();
}

hipError_t launch_resample(const ModelDev* Md, const RunDev& R, long long total, double logZ, long long n_out,
                           double* cum, int* idx, double* theta, hipStream_t st) {
  if (total <= 0 || n_out <= 0) return hipSuccess;
  double* u0 = cum + total;
  hipLaunchKernelGGL(k_resample_cum, dim3(1), dim3(1024), 0, st, R, total, logZ, cum, u0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_resample_pick, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, st, Md, R, total, cum,
                     u0, n_out, idx, theta);
  return hipGetLastError();
}

hipError_t launch_samples(const ModelDev* Md, const RunDev& R, long long total, double logZ, double* theta,
                          double* logl, double* logw, hipStream_t st) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_samples, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, Md, R, logZ, theta, logl,
                     logw);
  return hipGetLastError();
}

}  // namespace ns
