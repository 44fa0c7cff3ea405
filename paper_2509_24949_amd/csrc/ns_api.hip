// Host runtime of libns: argument validation, device memory of a run, the
// C ABI declared in include/ns.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include "../../include/ns.h"
#include "ns_runtime.h"

using namespace ns;

namespace ns {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int validate_and_model(const ns_problem* P, ModelDev* M) {
  if (!P) return fail(NS_E_ARG, "problem is NULL");
  memset(M, 0, sizeof(*M));
  if (P->n_dim < 1 || P->n_dim > MAX_DIM) return fail(NS_E_ARG, "n_dim must be in [1, %d]", MAX_DIM);
  if (P->likelihood < NS_LIKE_FULL || P->likelihood > NS_LIKE_GAUSS) return fail(NS_E_ARG, "unknown likelihood form");
  if (!P->prior_kind || !P->prior_lo || !P->prior_hi) return fail(NS_E_ARG, "prior arrays are NULL");
  M->likelihood = P->likelihood;
  M->n_dim = P->n_dim;
  for (int i = 0; i < P->n_dim; ++i) {
    const int k = P->prior_kind[i];
    const double lo = P->prior_lo[i], hi = P->prior_hi[i];
    if (!(lo <= hi) || !isfinite(lo) || !isfinite(hi)) return fail(NS_E_ARG, "prior %d: need finite lo <= hi", i);
    M->prior.kind[i] = k;
    M->prior.lo[i] = lo;
    M->prior.hi[i] = hi;
    switch (k) {
      case NS_PRIOR_UNIFORM: M->prior.a[i] = lo; M->prior.b[i] = hi - lo; break;
      case NS_PRIOR_COS:
        if (lo < 0.0 || hi > PI) return fail(NS_E_ARG, "prior %d: COS needs 0 <= lo <= hi <= pi", i);
        M->prior.a[i] = cos(lo); M->prior.b[i] = cos(hi) - cos(lo); break;
      case NS_PRIOR_SIN:
        if (lo < -0.5 * PI || hi > 0.5 * PI) return fail(NS_E_ARG, "prior %d: SIN needs -pi/2 <= lo <= hi <= pi/2", i);
        M->prior.a[i] = sin(lo); M->prior.b[i] = sin(hi) - sin(lo); break;
      case NS_PRIOR_VOLUME:
        if (lo < 0.0) return fail(NS_E_ARG, "prior %d: VOLUME needs lo >= 0", i);
        M->prior.a[i] = lo * lo * lo; M->prior.b[i] = hi * hi * hi - lo * lo * lo; break;
      default: return fail(NS_E_ARG, "prior %d: unknown kind %d", i, k);
    }
  }
  if (P->periodic) {
    for (int i = 0; i < P->n_dim; ++i) {
      if (P->periodic[i] != 0 && P->periodic[i] != 1) return fail(NS_E_ARG, "periodic[%d] must be 0 or 1", i);
      if (P->periodic[i] && P->prior_kind[i] != NS_PRIOR_UNIFORM)
        return fail(NS_E_ARG, "prior %d: a periodic coordinate needs a UNIFORM prior", i);
      if (P->periodic[i]) M->periodic |= 1u << i;
    }
  }
  if (P->likelihood == NS_LIKE_GAUSS) {
    if (!P->gauss_mu || !(P->gauss_sigma > 0.0)) return fail(NS_E_ARG, "Gaussian likelihood needs mu and sigma > 0");
    for (int i = 0; i < P->n_dim; ++i) M->gauss_mu[i] = P->gauss_mu[i];
    const double s = P->gauss_sigma;
    M->gauss_inv2s2 = 1.0 / (2.0 * s * s);
    M->gauss_norm = -0.5 * P->n_dim * log(2.0 * PI * s * s);
    M->n_det = 1;
    M->n_bins = 0;
    return NS_OK;
  }
  if (P->model != NS_MODEL_TF2_4P && P->model != NS_MODEL_TF2_11P && P->model != NS_MODEL_TF2_11P_SO)
    return fail(NS_E_ARG, "unknown waveform model");
  M->model = P->model;
  if (P->model == NS_MODEL_TF2_4P && (P->n_dim != 4 || P->n_det != 1))
    return fail(NS_E_ARG, "TF2_4P needs n_dim = 4 and n_det = 1");
  if (P->model != NS_MODEL_TF2_4P && (P->n_dim != 11 || P->n_det < 1 || P->n_det > MAX_DET))
    return fail(NS_E_ARG, "TF2_11P needs n_dim = 11 and 1 <= n_det <= %d", MAX_DET);
  if (!(P->f_lo > 0.0) || !(P->df > 0.0) || P->n_bins < 2) return fail(NS_E_ARG, "grid needs f_lo > 0, df > 0, n_bins >= 2");
  if (!P->data_re || !P->data_im || !P->psd) return fail(NS_E_ARG, "data and psd arrays are NULL");
  for (long i = 0; i < (long)P->n_det * P->n_bins; ++i)
    if (!(P->psd[i] > 0.0) || !isfinite(P->data_re[i]) || !isfinite(P->data_im[i]))
      return fail(NS_E_ARG, "psd must be positive and data finite (index %ld)", i);
  M->n_det = P->n_det;
  M->n_bins = P->n_bins;
  M->f_lo = P->f_lo;
  M->df = P->df;
  M->inv_df = 1.0 / P->df;
  M->gmst = P->gmst;
  // the largest f_ISCO over the prior box bounds the active bins
  double mc_min = P->prior_lo[0], eta_max;
  if (!(mc_min > 0.0)) return fail(NS_E_ARG, "chirp-mass prior must be positive");
  if (P->model == NS_MODEL_TF2_4P) {
    if (!(P->prior_lo[1] > 0.0) || P->prior_hi[1] > 0.25) return fail(NS_E_ARG, "eta prior must lie in (0, 0.25]");
    if (!(P->fixed_dist_mpc > 0.0)) return fail(NS_E_ARG, "fixed_dist_mpc must be positive");
    eta_max = P->prior_hi[1];
    M->fixed_dist_s = P->fixed_dist_mpc * MPC_S;
  } else {
    if (!(P->prior_lo[1] > 0.0) || P->prior_hi[1] > 1.0) return fail(NS_E_ARG, "mass-ratio prior must lie in (0, 1]");
    if (!(P->prior_lo[4] > 0.0)) return fail(NS_E_ARG, "distance prior must be positive");
    if (!P->det_geom) return fail(NS_E_ARG, "det_geom is NULL");
    const double q = P->prior_hi[1];
    eta_max = q / ((1.0 + q) * (1.0 + q));
    for (int d = 0; d < P->n_det; ++d) {
      const double* g = P->det_geom + 9 * d;
      const double* x = g + 3;
      const double* y = g + 6;
      double* D = M->det[d].D;
      D[0] = 0.5 * (x[0] * x[0] - y[0] * y[0]);
      D[1] = 0.5 * (x[0] * x[1] - y[0] * y[1]);
      D[2] = 0.5 * (x[0] * x[2] - y[0] * y[2]);
      D[3] = 0.5 * (x[1] * x[1] - y[1] * y[1]);
      D[4] = 0.5 * (x[1] * x[2] - y[1] * y[2]);
      D[5] = 0.5 * (x[2] * x[2] - y[2] * y[2]);
      for (int i = 0; i < 3; ++i) M->det[d].r_c[i] = g[i] / C_SI;
    }
  }
  // prior kinds each coordinate of the model supports
  for (int i = 0; i < P->n_dim; ++i) {
    const int k = P->prior_kind[i];
    bool ok = (k == NS_PRIOR_UNIFORM);
    if (P->model != NS_MODEL_TF2_4P && i == 4) ok = ok || k == NS_PRIOR_VOLUME;
    if (P->model != NS_MODEL_TF2_4P && i == 5) ok = ok || k == NS_PRIOR_COS;
    if (P->model != NS_MODEL_TF2_4P && i == 8) ok = ok || k == NS_PRIOR_SIN;
    if (!ok) return fail(NS_E_ARG, "prior %d: kind %d is not supported for this model coordinate", i, k);
  }
  const double m_min = mc_min * TSUN_S * pow(eta_max, -0.6);
  const double f_max = 1.0 / (pow(6.0, 1.5) * PI * m_min) * (1.0 + 1e-9);
  const double kk = floor((f_max - P->f_lo) / P->df) + 2.0;
  M->k_lim = (int)std::min<double>((double)P->n_bins, std::max(0.0, kk));
  if (P->likelihood == NS_LIKE_RB) {
    if (P->rb_n_bins < 1 || P->rb_n_bins >= P->n_bins || P->rb_n_bins > 1024)
      return fail(NS_E_ARG, "rb_n_bins must be in [1, min(n_bins - 1, 1024)]");
    if (!P->rb_fiducial) return fail(NS_E_ARG, "rb_fiducial is NULL");
    const double* th = P->rb_fiducial;
    for (int i = 0; i < P->n_dim; ++i)
      if (!isfinite(th[i])) return fail(NS_E_ARG, "rb_fiducial[%d] is not finite", i);
    if (!(th[0] > 0.0)) return fail(NS_E_ARG, "fiducial chirp mass must be positive");
    if (P->model == NS_MODEL_TF2_4P && !(th[1] > 0.0 && th[1] <= 0.25)) return fail(NS_E_ARG, "fiducial eta must lie in (0, 0.25]");
    if (P->model != NS_MODEL_TF2_4P && !(th[1] > 0.0 && th[1] <= 1.0 && th[4] > 0.0))
      return fail(NS_E_ARG, "fiducial needs q in (0, 1] and a positive distance");
  }
  return NS_OK;
}

int validate_opts(const ns_opts* o) {
  if (!o) return fail(NS_E_ARG, "opts is NULL");
  if (o->n_live < 2 || o->n_live > 16384) return fail(NS_E_ARG, "n_live must be in [2, 16384]");
  if (o->n_delete < 1 || o->n_delete >= o->n_live) return fail(NS_E_ARG, "n_delete must be in [1, n_live - 1]");
  if (o->n_steps < 1) return fail(NS_E_ARG, "n_steps must be >= 1");
  if (!(o->slice_width > 0.0)) return fail(NS_E_ARG, "slice_width must be > 0");
  if (o->max_stepout < 1 || o->max_shrink < 1) return fail(NS_E_ARG, "max_stepout and max_shrink must be >= 1");
  if (o->max_iter < 1) return fail(NS_E_ARG, "max_iter must be >= 1");
  if (o->precision != NS_FP64 && o->precision != NS_MIXED) return fail(NS_E_ARG, "precision must be NS_FP64 or NS_MIXED");
  if (o->kernel != NS_KERNEL_SLICE && o->kernel != NS_KERNEL_WALK)
    return fail(NS_E_ARG, "kernel must be NS_KERNEL_SLICE or NS_KERNEL_WALK");
  if (o->kernel == NS_KERNEL_WALK) {
    if (o->n_live - o->n_delete < 2) return fail(NS_E_ARG, "the random walk needs n_live - n_delete >= 2");
    if (o->walk_accept < 1 || o->walk_max < 1 || o->walk_max > (1 << 20))
      return fail(NS_E_ARG, "walk_accept must be >= 1 and walk_max in [1, 2^20]");
  }
  if (o->count_moves != 0 && o->count_moves != 1) return fail(NS_E_ARG, "count_moves must be 0 or 1");
  return NS_OK;
}

int sync_state(ns_run* r) {
  HIP_OK(hipMemcpyAsync(r->h_state, r->R.state, sizeof(DevState), hipMemcpyDeviceToHost, r->st));
  HIP_OK(hipStreamSynchronize(r->st));
  return NS_OK;
}

namespace {
size_t rounded(size_t bytes) { return (std::max<size_t>(bytes, 1) + 4095) / 4096 * 4096; }
}  // namespace

void run_footprint(const ns_problem* P, const ns_opts* O, size_t* resident, size_t* transient) {
  const size_t n = O->n_live, k = O->n_delete, d = P->n_dim;
  const size_t cap = (size_t)O->max_iter * k;
  size_t b = rounded(sizeof(ModelDev)) + rounded(sizeof(DevState)) + rounded(n * d * 8) + rounded(n * 8) +
             2 * rounded(n * 4) + 2 * rounded(k * 4) + rounded(d * d * 8) + 2 * rounded(k * 4) + rounded(k * 8) +
             rounded(cap * d * 8) + 3 * rounded(cap * 8) + 3 * rounded(cap * 4) + 2 * rounded(k * 4) +
             rounded((size_t)O->max_iter * sizeof(IterRec));
  size_t t = 0;
  if (P->likelihood != NS_LIKE_GAUSS) {
    const size_t nb = P->n_bins, nbd = (size_t)P->n_det * P->n_bins;
    b += 4 * rounded(nb * 8) + rounded(nbd * 16) + rounded(nbd * 8);
    if (O->precision == NS_MIXED && P->likelihood == NS_LIKE_FULL) b += rounded(nbd * 8);
    if (P->likelihood == NS_LIKE_RB) {
      const size_t q = std::max(P->rb_n_bins, 1), ne = q + 1, nbin = (size_t)P->n_det * q;
      b += rounded(ne * 4) + 4 * rounded(ne * 8) + rounded((size_t)P->n_det * ne * 8) + 2 * rounded(q * 8) +
           rounded((size_t)P->n_det * 16) + 2 * rounded(nbin * 16) + 2 * rounded(nbin * 8) + 2 * rounded(nbd * 16) +
           2 * rounded(nbd * 8) + rounded(MAX_DIM * 8);
      if (O->precision == NS_MIXED) b += 2 * rounded(nbin * 8) + 2 * rounded(nbin * 4);
      b += rounded(rb_edge_record_doubles((int)q, P->n_det, O->precision == NS_MIXED) * 8);
    }
    t = rounded(4 * nbd * 8);
  }
  *resident = b;
  *transient = t;
}

int run_create(ns_run** out, const ns_problem* P, const ns_opts* O, hipStream_t stream, bool packed) {
  if (!out) return fail(NS_E_ARG, "out is NULL");
  *out = nullptr;
  ModelDev M;
  int rc = validate_and_model(P, &M);
  if (rc) return rc;
  if ((rc = validate_opts(O))) return rc;
  ns_run* r = new (std::nothrow) ns_run();
  if (!r) return fail(NS_E_OOM, "host allocation failed");
  r->prob.own(*P);
  r->opts = *O;
  M.mixed = (O->precision == NS_MIXED && M.likelihood != NS_LIKE_GAUSS) ? 1 : 0;
  M.dw_scale = 1.0;
  if (M.mixed && M.likelihood == NS_LIKE_FULL) {
    // a power of two that brings the largest whitened data value near 1 (exact in float)
    double mx = 0.0;
    for (int d = 0; d < M.n_det; ++d)
      for (int k = 0; k < M.n_bins; ++k) {
        const size_t o = (size_t)d * M.n_bins + k;
        const double f = M.f_lo + k * M.df;
        const double a = 4.0 * M.df * pow(f, -7.0 / 6.0) / P->psd[o];
        mx = std::max(mx, a * std::max(fabs(P->data_re[o]), fabs(P->data_im[o])));
      }
    if (mx > 0.0 && isfinite(mx)) M.dw_scale = ldexp(1.0, -ilogb(mx));
  }
  r->M = M;
  r->st = stream;
  r->packed = packed;
  const int n = O->n_live, k = O->n_delete, d = P->n_dim;
  RunDev& R = r->R;
  R.n = n; R.k = k; R.d = d; R.m = O->n_steps;
  R.width = O->slice_width;
  R.max_stepout = O->max_stepout;
  R.max_shrink = O->max_shrink;
  R.log_term = O->term_frac > 0.0 ? log(O->term_frac) : -__builtin_inf();
  R.key0 = O->seed;
  R.key1 = O->run_id;
  R.cap = (long long)O->max_iter * k;
  R.kernel = O->kernel;
  R.walk_accept = O->walk_accept;
  R.walk_max = O->walk_max;
  R.move_counts = (!packed && O->kernel == NS_KERNEL_SLICE && O->count_moves) ? 1 : 0;
  auto cleanup = [&](int code) { delete r; return code; };
  DevMem& mem = r->mem;
#define ALLOC(ptr, count) \
  if (mem.alloc(&(ptr), (count)) != hipSuccess) return cleanup(fail(NS_E_OOM, "hipMalloc failed for " #ptr))
  ALLOC(r->Md, 1);
  ALLOC(R.state, 1);
  ALLOC(R.u, (size_t)n * d);
  ALLOC(R.lam, n);
  ALLOC(R.rank, n);
  ALLOC(R.dead, k);
  ALLOC(R.surv, n);
  ALLOC(R.start, k);
  ALLOC(R.chol, (size_t)d * d);
  ALLOC(R.probes, k);
  ALLOC(R.acc, k);
  ALLOC(R.bins, k);
  ALLOC(R.nso, k);
  ALLOC(R.nsh, k);
  R.trace_cap = O->max_iter;
  ALLOC(R.trace, (size_t)O->max_iter);
  ALLOC(R.du, (size_t)R.cap * d);
  ALLOC(R.dlam, R.cap);
  ALLOC(R.dlogx, R.cap);
  ALLOC(R.dlogw, R.cap);
  ALLOC(R.diter, R.cap);
  ALLOC(R.dslot, R.cap);
  ALLOC(R.dnlive, R.cap);
  if (hipHostMalloc((void**)&r->h_state, sizeof(DevState), hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(NS_E_OOM, "pinned allocation failed"));

  hipError_t e = hipMemcpyAsync(r->Md, &r->M, sizeof(ModelDev), hipMemcpyHostToDevice, r->st);
  if (e != hipSuccess) return cleanup(fail(NS_E_HIP, "copying the model: %s", hipGetErrorString(e)));
  if (M.likelihood != NS_LIKE_GAUSS) {
    const size_t nbd = (size_t)M.n_det * M.n_bins;
    double *f, *f13, *lnf3, *fm53, *hpre, *dre, *dim, *psd, *scratch;
    double2* dw;
    ALLOC(f, M.n_bins); ALLOC(f13, M.n_bins); ALLOC(lnf3, M.n_bins); ALLOC(fm53, M.n_bins);
    ALLOC(dw, nbd); ALLOC(hpre, nbd);
    std::vector<void*> tmp;
    double* stage = nullptr;
    if (hipMalloc((void**)&stage, 4 * nbd * sizeof(double)) != hipSuccess)
      return cleanup(fail(NS_E_OOM, "hipMalloc failed for staging"));
    dre = stage; dim = stage + nbd; psd = stage + 2 * nbd; scratch = stage + 3 * nbd;
    e = hipMemcpyAsync(dre, P->data_re, nbd * sizeof(double), hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess) e = hipMemcpyAsync(dim, P->data_im, nbd * sizeof(double), hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess) e = hipMemcpyAsync(psd, P->psd, nbd * sizeof(double), hipMemcpyHostToDevice, r->st);
    double* d_noise = nullptr;
    ALLOC(d_noise, 1);
    if (e == hipSuccess)
      e = launch_build_tables(M, r->Md, dre, dim, psd, f, f13, lnf3, fm53, dw, hpre, scratch, r->st);
    if (e == hipSuccess) e = launch_noise_loglike(dre, dim, psd, (long)nbd, M.df, d_noise, r->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&r->noise_loglike, d_noise, sizeof(double), hipMemcpyDeviceToHost, r->st);
    if (e == hipSuccess) e = hipStreamSynchronize(r->st);
    r->T.f = f; r->T.f13 = f13; r->T.lnf3 = lnf3; r->T.fm53 = fm53; r->T.dw = dw; r->T.hpre = hpre;
    if (e == hipSuccess && M.mixed && M.likelihood == NS_LIKE_FULL) {
      float2* dw32;
      if (mem.alloc(&dw32, nbd) != hipSuccess) {
        (void)hipFree(stage);
        return cleanup(fail(NS_E_OOM, "hipMalloc failed for the float data table"));
      }
      e = launch_to_float(dw, dw32, nbd, M.dw_scale, r->st);
      r->T.dw32 = dw32;
    }
    if (e == hipSuccess && M.likelihood == NS_LIKE_RB) {
      // relative binning: edges, fiducial phases, summary sums (scratch holds the weights 4 df f^(-7/3) / S)
      const int nb = P->rb_n_bins;
      const size_t ne = nb + 1, nbin = (size_t)M.n_det * nb;
      RBBuffers B{};
      double* th = nullptr;
      bool ok = mem.alloc(&B.edge, ne) == hipSuccess && mem.alloc(&B.fe, ne) == hipSuccess &&
                mem.alloc(&B.fe13, ne) == hipSuccess && mem.alloc(&B.lnfe3, ne) == hipSuccess &&
                mem.alloc(&B.fem53, ne) == hipSuccess && mem.alloc(&B.phi0, (size_t)M.n_det * ne) == hipSuccess &&
                mem.alloc(&B.fm, nb) == hipSuccess && mem.alloc(&B.inv_w, nb) == hipSuccess &&
                mem.alloc(&B.g0, M.n_det) == hipSuccess && mem.alloc(&B.A0, nbin) == hipSuccess &&
                mem.alloc(&B.A1, nbin) == hipSuccess && mem.alloc(&B.B0, nbin) == hipSuccess &&
                mem.alloc(&B.B1, nbin) == hipSuccess && mem.alloc(&B.cA0, nbd) == hipSuccess &&
                mem.alloc(&B.cA1, nbd) == hipSuccess && mem.alloc(&B.cB0, nbd) == hipSuccess &&
                mem.alloc(&B.cB1, nbd) == hipSuccess && mem.alloc(&th, MAX_DIM) == hipSuccess;
      if (!ok) {
        (void)hipFree(stage);
        return cleanup(fail(NS_E_OOM, "hipMalloc failed for relative-binning tables"));
      }
      std::vector<int> edges(ne);
      e = hipMemcpyAsync(th, P->rb_fiducial, P->n_dim * sizeof(double), hipMemcpyHostToDevice, r->st);
      if (e == hipSuccess) e = launch_build_rb_edges(r->Md, nb, B, r->st);
      if (e == hipSuccess) e = hipMemcpyAsync(edges.data(), B.edge, ne * sizeof(int), hipMemcpyDeviceToHost, r->st);
      if (e == hipSuccess) e = hipStreamSynchronize(r->st);
      if (e == hipSuccess) {
        for (int i = 0; i < nb; ++i)
          if (edges[i + 1] <= edges[i]) {
            (void)hipFree(stage);
            return cleanup(fail(NS_E_ARG, "rb_n_bins = %d gives empty coarse bins on this grid (edge %d)", nb, i + 1));
          }
      }
      if (e == hipSuccess) e = launch_build_rb_sums(M, r->Md, r->T, scratch, th, nb, B, r->st);
      if (e == hipSuccess && M.mixed) {
        if (mem.alloc(&B.A0f, nbin) != hipSuccess || mem.alloc(&B.A1f, nbin) != hipSuccess ||
            mem.alloc(&B.B0f, nbin) != hipSuccess || mem.alloc(&B.B1f, nbin) != hipSuccess) {
          (void)hipFree(stage);
          return cleanup(fail(NS_E_OOM, "hipMalloc failed for the float bin sums"));
        }
        e = launch_to_float(B.A0, B.A0f, nbin, 1.0, r->st);
        if (e == hipSuccess) e = launch_to_float(B.A1, B.A1f, nbin, 1.0, r->st);
        if (e == hipSuccess) e = launch_to_float(B.B0, B.B0f, nbin, 1.0, r->st);
        if (e == hipSuccess) e = launch_to_float(B.B1, B.B1f, nbin, 1.0, r->st);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(r->st);
      RBTables& RB = r->RB;
      RB.nb = nb;
      RB.edge = B.edge; RB.fe = B.fe; RB.fe13 = B.fe13; RB.lnfe3 = B.lnfe3; RB.fem53 = B.fem53;
      RB.phi0 = B.phi0; RB.g0 = B.g0; RB.fm = B.fm; RB.inv_w = B.inv_w;
      RB.A0 = B.A0; RB.A1 = B.A1; RB.B0 = B.B0; RB.B1 = B.B1;
      RB.cA0 = B.cA0; RB.cA1 = B.cA1; RB.cB0 = B.cB0; RB.cB1 = B.cB1;
      RB.A0f = B.A0f; RB.A1f = B.A1f; RB.B0f = B.B0f; RB.B1f = B.B1f;
      if (e == hipSuccess) {
        if (mem.alloc(&B.erec, rb_edge_record_doubles(nb, M.n_det, M.mixed != 0)) != hipSuccess) {
          (void)hipFree(stage);
          return cleanup(fail(NS_E_OOM, "hipMalloc failed for the edge records"));
        }
        e = launch_build_rb_edge_records(M, RB, B.erec, r->st);
        if (e == hipSuccess) e = hipStreamSynchronize(r->st);
        RB.erec = B.erec;
      }
    }
    (void)hipFree(stage);
    if (e != hipSuccess) return cleanup(fail(NS_E_HIP, "building likelihood tables: %s", hipGetErrorString(e)));
  }
#undef ALLOC
  if (packed) (void)configure_slice_packed(r->M, r->RB.nb, &r->C);
  else (void)configure_slice(r->M, r->RB.nb, R.k, R.move_counts != 0, &r->C);
  DevState s0{};
  s0.logX = 0.0;
  s0.logZ = -__builtin_inf();
  s0.H = 0.0;
  s0.lstar = -__builtin_inf();
  s0.n_dead = 0;
  s0.n_evals = n;
  s0.iter = 0;
  s0.done = 0;
  s0.walk_len = O->kernel == NS_KERNEL_WALK ? std::min(O->walk_accept, O->walk_max) : 0;
  *r->h_state = s0;
  e = hipMemcpyAsync(R.state, r->h_state, sizeof(DevState), hipMemcpyHostToDevice, r->st);
  if (e == hipSuccess) e = launch_init_live(R, r->st);
  if (e == hipSuccess) e = launch_loglike(r->M, r->Md, r->T, r->RB, R.u, n, R.lam, nullptr, nullptr, r->st);
  if (e == hipSuccess) e = hipStreamSynchronize(r->st);
  if (e != hipSuccess) return cleanup(fail(NS_E_HIP, "initial population: %s", hipGetErrorString(e)));
  // the device of the run and its no-allocation scratch, looked up once per
  // device (the runtime is initialised by now)
  Probe* scratch_addr = nullptr;
  e = hipGetDevice(&r->device);
  if (e == hipSuccess) e = noalloc_probe_scratch(r->device, &scratch_addr);
  if (e != hipSuccess) return cleanup(fail(NS_E_HIP, "device set-up: %s", hipGetErrorString(e)));
  *out = r;
  return NS_OK;
}

}  // namespace ns

extern "C" {

const char* ns_last_error(void) { return g_err.c_str(); }

int ns_init(ns_run** out, const ns_problem* P, const ns_opts* O, void* stream) {
  TraceRange range_("ns_init");
  return run_create(out, P, O, static_cast<hipStream_t>(stream), false);
}

int ns_step_async(ns_run* r, int n_iters) {
  TraceRange range_("ns_step_async");
  if (!r) return fail(NS_E_ARG, "run is NULL");
  if (n_iters < 0) return fail(NS_E_ARG, "n_iters must be >= 0");
  for (int i = 0; i < n_iters; ++i) {
    hipEvent_t* ev = nullptr;
    if (r->profiling) {
      std::array<hipEvent_t, 5> a{};
      for (auto& e : a) HIP_OK(hipEventCreate(&e));
      r->events.push_back(a);
      ev = r->events.back().data();
    }
    HIP_OK(launch_iteration(r->M, r->Md, r->T, r->RB, r->R, r->C, r->st, ev));
  }
  return NS_OK;
}

int ns_profile(ns_run* r, int enable) {
  if (!r) return fail(NS_E_ARG, "run is NULL");
  HIP_OK(hipStreamSynchronize(r->st));
  r->release_events();
  r->profiling = enable != 0;
  return NS_OK;
}

int ns_stats(ns_run* r, ns_stats_t* out) {
  if (!r || !out) return fail(NS_E_ARG, "NULL argument");
  int rc = sync_state(r);
  if (rc) return rc;
  memset(out, 0, sizeof(*out));
  for (auto& a : r->events) {
    float t[4];
    for (int i = 0; i < 4; ++i) HIP_OK(hipEventElapsedTime(&t[i], a[i], a[i + 1]));
    out->ms_select += t[0];
    out->ms_prep += t[1];
    out->ms_slice += t[2];
    out->ms_term += t[3];
  }
  out->iterations = (long)r->events.size();
  out->evals = r->h_state->n_evals;
  out->bin_terms = r->h_state->n_bin_terms;
  out->slice_threads = r->C.slice_threads;
  out->lds_tables = r->C.lds_tables ? 1 : 0;
  return NS_OK;
}

int ns_trace(ns_run* r, long cap, ns_iter_t* out, long* n_out) {
  if (!r || !n_out) return fail(NS_E_ARG, "NULL argument");
  int rc = sync_state(r);
  if (rc) return rc;
  const long n = std::min<long>(r->h_state->iter, r->R.trace_cap);
  *n_out = n;
  if (!out) return NS_OK;
  if (cap < n) return fail(NS_E_CAPACITY, "%ld iterations recorded, cap is %ld", n, cap);
  if (n) {
    HIP_OK(hipMemcpyAsync(out, r->R.trace, (size_t)n * sizeof(IterRec), hipMemcpyDeviceToHost, r->st));
    HIP_OK(hipStreamSynchronize(r->st));
  }
  return NS_OK;
}

int ns_step(ns_run* r, int max_iters, int* done) {
  TraceRange range_("ns_step");
  int rc = ns_step_async(r, max_iters);
  if (rc) return rc;
  if ((rc = sync_state(r))) return rc;
  if (done) *done = r->h_state->done != 0;
  return NS_OK;
}

int ns_state(ns_run* r, double* logX, double* logZ, double* H, int* iter, long* n_dead, long* n_evals, int* done) {
  if (!r) return fail(NS_E_ARG, "run is NULL");
  int rc = sync_state(r);
  if (rc) return rc;
  const DevState& s = *r->h_state;
  if (logX) *logX = s.logX;
  if (logZ) *logZ = s.logZ;
  if (H) *H = s.H;
  if (iter) *iter = s.iter;
  if (n_dead) *n_dead = (long)s.n_dead;
  if (n_evals) *n_evals = (long)s.n_evals;
  if (done) *done = s.done;
  return NS_OK;
}

int ns_logZ(ns_run* r, int n_sim, double* logZ, double* sigma_sim, double* sigma_h, double* ess) {
  TraceRange range_("ns_logZ");
  if (!r) return fail(NS_E_ARG, "run is NULL");
  if (n_sim < 0 || n_sim > 100000) return fail(NS_E_ARG, "n_sim must be in [0, 100000]");
  const int ns_ = n_sim >= 2 ? n_sim : 0;
  double* dout = nullptr;
  HIP_OK(hipMalloc((void**)&dout, (3 + ns_) * sizeof(double)));
  std::vector<double> h(3 + ns_);
  hipError_t e = launch_final(r->R, ns_, dout, r->st);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), dout, h.size() * sizeof(double), hipMemcpyDeviceToHost, r->st);
  if (e == hipSuccess) e = hipStreamSynchronize(r->st);
  (void)hipFree(dout);
  if (e != hipSuccess) return fail(NS_E_HIP, "finalisation: %s", hipGetErrorString(e));
  if (logZ) *logZ = h[0];
  if (sigma_h) *sigma_h = sqrt(h[1] > 0.0 ? h[1] / r->R.n : 0.0);
  if (ess) *ess = h[2];
  if (sigma_sim) {
    double sd = 0.0;
    if (ns_ >= 2) {
      double m = 0.0;
      for (int i = 0; i < ns_; ++i) m += h[3 + i];
      m /= ns_;
      for (int i = 0; i < ns_; ++i) sd += (h[3 + i] - m) * (h[3 + i] - m);
      sd = sqrt(sd / (ns_ - 1));
    }
    *sigma_sim = sd;
  }
  return NS_OK;
}

int ns_samples(ns_run* r, long cap, double* theta, double* logl, double* logw, long* n_out) {
  TraceRange range_("ns_samples");
  if (!r) return fail(NS_E_ARG, "run is NULL");
  int rc = sync_state(r);
  if (rc) return rc;
  const long long total = r->h_state->n_dead + r->R.n;
  if (n_out) *n_out = (long)total;
  if (cap < total) return fail(NS_E_CAPACITY, "need %lld samples, cap is %ld", total, cap);
  double lz = 0.0;
  if ((rc = ns_logZ(r, 0, &lz, nullptr, nullptr, nullptr))) return rc;
  const int d = r->R.d;
  double *dth = nullptr, *dl = nullptr, *dw = nullptr;
  HIP_OK(hipMalloc((void**)&dth, std::max<long long>(1, total * d) * sizeof(double)));
  hipError_t e = hipMalloc((void**)&dl, std::max<long long>(1, total) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&dw, std::max<long long>(1, total) * sizeof(double));
  if (e == hipSuccess) e = launch_samples(r->Md, r->R, total, lz, dth, dl, dw, r->st);
  if (e == hipSuccess && theta) e = hipMemcpyAsync(theta, dth, total * d * sizeof(double), hipMemcpyDeviceToHost, r->st);
  if (e == hipSuccess && logl) e = hipMemcpyAsync(logl, dl, total * sizeof(double), hipMemcpyDeviceToHost, r->st);
  if (e == hipSuccess && logw) e = hipMemcpyAsync(logw, dw, total * sizeof(double), hipMemcpyDeviceToHost, r->st);
  if (e == hipSuccess) e = hipStreamSynchronize(r->st);
  (void)hipFree(dth);
  (void)hipFree(dl);
  (void)hipFree(dw);
  if (e != hipSuccess) return fail(NS_E_HIP, "samples: %s", hipGetErrorString(e));
  return NS_OK;
}

int ns_resample(ns_run* r, long n_out, int* idx, double* theta) {
  TraceRange range_("ns_resample");
  if (!r) return fail(NS_E_ARG, "run is NULL");
  if (n_out < 1 || n_out > (1L << 30)) return fail(NS_E_ARG, "n_out must be in 1..2^30");
  int rc = sync_state(r);
  if (rc) return rc;
  const long long total = r->h_state->n_dead + r->R.n;
  double lz = 0.0;
  if ((rc = ns_logZ(r, 0, &lz, nullptr, nullptr, nullptr))) return rc;
  const int d = r->R.d;
  double *cum = nullptr, *dth = nullptr;
  int* di = nullptr;
  HIP_OK(hipMalloc((void**)&cum, (total + 1) * sizeof(double)));
  hipError_t e = hipMalloc((void**)&di, n_out * sizeof(int));
  if (e == hipSuccess && theta) e = hipMalloc((void**)&dth, (size_t)n_out * d * sizeof(double));
  if (e == hipSuccess) e = launch_resample(r->Md, r->R, total, lz, n_out, cum, di, dth, r->st);
  if (e == hipSuccess && idx) e = hipMemcpyAsync(idx, di, n_out * sizeof(int), hipMemcpyDeviceToHost, r->st);
  if (e == hipSuccess && theta)
    e = hipMemcpyAsync(theta, dth, (size_t)n_out * d * sizeof(double), hipMemcpyDeviceToHost, r->st);
  if (e == hipSuccess) e = hipStreamSynchronize(r->st);
  (void)hipFree(cum);
  (void)hipFree(di);
  (void)hipFree(dth);
  if (e != hipSuccess) return fail(NS_E_HIP, "resample: %s", hipGetErrorString(e));
  return NS_OK;
}

int ns_live(ns_run* r, double* u, double* logl) {
  if (!r) return fail(NS_E_ARG, "run is NULL");
  if (u) HIP_OK(hipMemcpyAsync(u, r->R.u, (size_t)r->R.n * r->R.d * sizeof(double), hipMemcpyDeviceToHost, r->st));
  if (logl) HIP_OK(hipMemcpyAsync(logl, r->R.lam, (size_t)r->R.n * sizeof(double), hipMemcpyDeviceToHost, r->st));
  HIP_OK(hipStreamSynchronize(r->st));
  return NS_OK;
}

int ns_dead(ns_run* r, long cap, double* u, double* logl, double* logx, double* logw, int* iter, int* slot,
            long* n_out) {
  if (!r) return fail(NS_E_ARG, "run is NULL");
  int rc = sync_state(r);
  if (rc) return rc;
  const long long nd = r->h_state->n_dead;
  if (n_out) *n_out = (long)nd;
  if (cap < nd) return fail(NS_E_CAPACITY, "need %lld dead points, cap is %ld", nd, cap);
  const RunDev& R = r->R;
  const size_t b = (size_t)nd * sizeof(double);
  if (nd > 0) {
    if (u) HIP_OK(hipMemcpyAsync(u, R.du, b * R.d, hipMemcpyDeviceToHost, r->st));
    if (logl) HIP_OK(hipMemcpyAsync(logl, R.dlam, b, hipMemcpyDeviceToHost, r->st));
    if (logx) HIP_OK(hipMemcpyAsync(logx, R.dlogx, b, hipMemcpyDeviceToHost, r->st));
    if (logw) HIP_OK(hipMemcpyAsync(logw, R.dlogw, b, hipMemcpyDeviceToHost, r->st));
    if (iter) HIP_OK(hipMemcpyAsync(iter, R.diter, (size_t)nd * sizeof(int), hipMemcpyDeviceToHost, r->st));
    if (slot) HIP_OK(hipMemcpyAsync(slot, R.dslot, (size_t)nd * sizeof(int), hipMemcpyDeviceToHost, r->st));
  }
  HIP_OK(hipStreamSynchronize(r->st));
  return NS_OK;
}

int ns_loglike(ns_run* r, const double* u_dev, long n, double* out_dev, int* terms_dev) {
  TraceRange range_("ns_loglike");
  if (!r) return fail(NS_E_ARG, "run is NULL");
  if (n < 0 || (n > 0 && (!u_dev || !out_dev))) return fail(NS_E_ARG, "bad batch arguments");
  const bool two_pass = r->M.likelihood == NS_LIKE_FULL;   // the full grid stores probe records
  if (two_pass && n > r->probe_cap) {
    HIP_OK(hipStreamSynchronize(r->st));   // the old buffer may still be read
    if (r->probe_buf) (void)hipFree(r->probe_buf);
    r->probe_buf = nullptr;
    r->probe_cap = 0;
    const long cap = std::max<long>(n, 4096);
    HIP_OK(hipMalloc((void**)&r->probe_buf, cap * sizeof(Probe)));
    r->probe_cap = cap;
  }
  HIP_OK(launch_loglike(r->M, r->Md, r->T, r->RB, u_dev, n, out_dev, terms_dev,
                        two_pass ? r->probe_buf : nullptr, r->st));
  return NS_OK;
}

int ns_loglike_noalloc(ns_run* r, const double* u_dev, long n, double* out_dev, int* terms_dev) {
  if (!r) return fail(NS_E_ARG, "run is NULL");
  if (n < 0 || (n > 0 && (!u_dev || !out_dev))) return fail(NS_E_ARG, "bad batch arguments");
  if (n > NS_LOGLIKE_NOALLOC_MAX)
    return fail(NS_E_ARG, "batch of %ld probes exceeds NS_LOGLIKE_NOALLOC_MAX (%d)", n, NS_LOGLIKE_NOALLOC_MAX);
  int cur = -1;
  HIP_OK(hipGetDevice(&cur));
  if (cur != r->device) return fail(NS_E_ARG, "the current device (%d) is not the run's (%d)", cur, r->device);
  const bool two_pass = r->M.likelihood == NS_LIKE_FULL;   // the full grid stores probe records
  Probe* buf = nullptr;
  if (two_pass) HIP_OK(noalloc_probe_scratch(r->device, &buf));
  HIP_OK(launch_loglike(r->M, r->Md, r->T, r->RB, u_dev, n, out_dev, terms_dev, buf, r->st));
  return NS_OK;
}

int ns_waveform(const ns_problem* P, const double* theta, int det, int apply_cut, double* h_re, double* h_im,
                void* stream) {
  if (!P || !theta || !h_re || !h_im) return fail(NS_E_ARG, "NULL argument");
  ns_problem q = *P;
  q.likelihood = NS_LIKE_FULL;
  ModelDev M;
  // data are not read by the waveform; validate the rest with a zero stand-in
  std::vector<double> zero, one;
  if (!P->data_re || !P->data_im || !P->psd) {
    zero.assign((size_t)std::max(P->n_det, 1) * std::max(P->n_bins, 1), 0.0);
    one.assign(zero.size(), 1.0);
    q.data_re = zero.data(); q.data_im = zero.data(); q.psd = one.data();
  }
  int rc = validate_and_model(&q, &M);
  if (rc) return rc;
  if (det < 0 || det >= M.n_det) return fail(NS_E_ARG, "det out of range");
  M.k_lim = M.n_bins;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double *dth = nullptr, *dre = nullptr, *dim = nullptr;
  ModelDev* Md = nullptr;
  HIP_OK(hipMalloc((void**)&dth, MAX_DIM * sizeof(double)));
  hipError_t e = hipMalloc((void**)&dre, M.n_bins * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&dim, M.n_bins * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&Md, sizeof(ModelDev));
  if (e == hipSuccess) e = hipMemcpyAsync(Md, &M, sizeof(ModelDev), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dth, theta, P->n_dim * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_waveform(M, Md, dth, det, apply_cut, dre, dim, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h_re, dre, M.n_bins * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h_im, dim, M.n_bins * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dth);
  (void)hipFree(dre);
  (void)hipFree(dim);
  (void)hipFree(Md);
  if (e != hipSuccess) return fail(NS_E_HIP, "waveform: %s", hipGetErrorString(e));
  return NS_OK;
}

int ns_select(const double* logl_dev, int n, int k, int* dead_dev, double* lstar_dev, void* stream) {
  if (!logl_dev || !dead_dev) return fail(NS_E_ARG, "NULL argument");
  if (n < 1 || n > 16384 || k < 1 || k > n) return fail(NS_E_ARG, "need 1 <= k <= n <= 16384");
  HIP_OK(launch_select(logl_dev, n, k, nullptr, dead_dev, lstar_dev, nullptr, static_cast<hipStream_t>(stream)));
  return NS_OK;
}

int ns_noise_loglike(ns_run* r, double* out) {
  if (!r || !out) return fail(NS_E_ARG, "NULL argument");
  if (r->M.likelihood == NS_LIKE_GAUSS) return fail(NS_E_STATE, "the Gaussian test likelihood has no noise model");
  *out = r->noise_loglike;
  return NS_OK;
}

}  // extern "C"

// The device's metrics record is the public one.
static_assert(sizeof(IterRec) == sizeof(ns_iter_t) && offsetof(IterRec, lstar) == offsetof(ns_iter_t, lstar) &&
                  offsetof(IterRec, probes) == offsetof(ns_iter_t, probes) &&
                  offsetof(IterRec, shrinks) == offsetof(ns_iter_t, shrinks) &&
                  offsetof(IterRec, hist) == offsetof(ns_iter_t, hist) && PROBE_HIST == NS_PROBE_HIST,
              "metrics record layout");

// ---- checkpoint format ------------------------------------------------------
namespace {

constexpr char kMagic[8] = {'N', 'S', 'R', 'U', 'N', 'v', '3', '\0'};

struct Writer {
  unsigned char* buf;
  size_t cap, n = 0;
  void raw(const void* p, size_t b) {
    if (buf && n + b <= cap) memcpy(buf + n, p, b);
    n += b;
  }
  template <typename T>
  void val(const T& v) { raw(&v, sizeof(T)); }
  template <typename T>
  void vec(const std::vector<T>& v) {
    val<uint64_t>(v.size());
    raw(v.data(), v.size() * sizeof(T));
  }
};

struct Reader {
  const unsigned char* buf;
  size_t size, n = 0;
  bool ok = true;
  void raw(void* p, size_t b) {
    if (!ok || b > size - n) { ok = false; return; }
    memcpy(p, buf + n, b);
    n += b;
  }
  template <typename T>
  T val() { T v{}; raw(&v, sizeof(T)); return v; }
  template <typename T>
  std::vector<T> vec(size_t max_count) {
    const uint64_t c = val<uint64_t>();
    std::vector<T> v;
    if (!ok || c > max_count || c * sizeof(T) > size - n) { ok = false; return v; }
    v.resize(c);
    raw(v.data(), c * sizeof(T));
    return v;
  }
};

// Problem scalars stored in a checkpoint (pointers are written as arrays).
struct ProblemScalars {
  int model, likelihood, n_dim, n_bins, n_det, rb_n_bins;
  double f_lo, df, gmst, fixed_dist_mpc, gauss_sigma;
};

}  // namespace

extern "C" {

int ns_save(ns_run* r, void* buf, size_t cap, size_t* n_out) {
  TraceRange range_("ns_save");
  if (!r) return fail(NS_E_ARG, "run is NULL");
  int rc = sync_state(r);
  if (rc) return rc;
  const RunDev& R = r->R;
  const DevState st = *r->h_state;
  const size_t nd = (size_t)st.n_dead;
  std::vector<double> u((size_t)R.n * R.d), lam(R.n), du(nd * R.d), dlam(nd), dlogx(nd), dlogw(nd);
  std::vector<int> diter(nd), dslot(nd), dnlive(nd);
  std::vector<IterRec> trace((size_t)std::min<long long>(st.iter, R.trace_cap));
  const bool fetch = buf != nullptr;
  Writer w{nullptr, 0};   // the first pass only measures
  const ns_problem& P = r->prob.P;
  ProblemScalars ps{P.model, P.likelihood, P.n_dim, P.n_bins, P.n_det, P.rb_n_bins,
                    P.f_lo, P.df, P.gmst, P.fixed_dist_mpc, P.gauss_sigma};
  // size first: the record is written only if it fits
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      if (!fetch || w.n > cap) break;
      HIP_OK(hipMemcpyAsync(u.data(), R.u, u.size() * sizeof(double), hipMemcpyDeviceToHost, r->st));
      HIP_OK(hipMemcpyAsync(lam.data(), R.lam, lam.size() * sizeof(double), hipMemcpyDeviceToHost, r->st));
      if (nd) {
        HIP_OK(hipMemcpyAsync(du.data(), R.du, du.size() * sizeof(double), hipMemcpyDeviceToHost, r->st));
        HIP_OK(hipMemcpyAsync(dlam.data(), R.dlam, nd * sizeof(double), hipMemcpyDeviceToHost, r->st));
        HIP_OK(hipMemcpyAsync(dlogx.data(), R.dlogx, nd * sizeof(double), hipMemcpyDeviceToHost, r->st));
        HIP_OK(hipMemcpyAsync(dlogw.data(), R.dlogw, nd * sizeof(double), hipMemcpyDeviceToHost, r->st));
        HIP_OK(hipMemcpyAsync(diter.data(), R.diter, nd * sizeof(int), hipMemcpyDeviceToHost, r->st));
        HIP_OK(hipMemcpyAsync(dslot.data(), R.dslot, nd * sizeof(int), hipMemcpyDeviceToHost, r->st));
        HIP_OK(hipMemcpyAsync(dnlive.data(), R.dnlive, nd * sizeof(int), hipMemcpyDeviceToHost, r->st));
      }
      if (!trace.empty())
        HIP_OK(hipMemcpyAsync(trace.data(), R.trace, trace.size() * sizeof(IterRec), hipMemcpyDeviceToHost, r->st));
      HIP_OK(hipStreamSynchronize(r->st));
      w = Writer{static_cast<unsigned char*>(buf), cap};
    }
    w.raw(kMagic, sizeof kMagic);
    w.val<int>(r->packed ? 1 : 0);
    w.val(ps);
    w.val(r->opts);
    w.vec(r->prob.kind);
    w.vec(r->prob.lo);
    w.vec(r->prob.hi);
    w.vec(r->prob.dre);
    w.vec(r->prob.dim);
    w.vec(r->prob.psd);
    w.vec(r->prob.geom);
    w.vec(r->prob.fid);
    w.vec(r->prob.mu);
    w.vec(r->prob.per);
    w.val(st);
    w.vec(u);
    w.vec(lam);
    w.vec(du);
    w.vec(dlam);
    w.vec(dlogx);
    w.vec(dlogw);
    w.vec(diter);
    w.vec(dslot);
    w.vec(dnlive);
    w.vec(trace);
  }
  if (n_out) *n_out = w.n;
  if (!buf || w.n > cap) return fail(NS_E_CAPACITY, "the checkpoint needs %zu bytes, cap is %zu", w.n, buf ? cap : 0);
  return NS_OK;
}

int ns_load(ns_run** out, const void* buf, size_t size, void* stream) {
  TraceRange range_("ns_load");
  if (!out || !buf) return fail(NS_E_ARG, "NULL argument");
  *out = nullptr;
  Reader rd{static_cast<const unsigned char*>(buf), size};
  char magic[8];
  rd.raw(magic, sizeof magic);
  if (!rd.ok || memcmp(magic, kMagic, sizeof magic) != 0) return fail(NS_E_ARG, "not a run checkpoint");
  const int packed = rd.val<int>();
  const ProblemScalars ps = rd.val<ProblemScalars>();
  const ns_opts O = rd.val<ns_opts>();
  if (!rd.ok) return fail(NS_E_ARG, "truncated checkpoint");
  const size_t big = size / sizeof(double) + 1;
  ProblemCopy pc;
  pc.kind = rd.vec<int>(MAX_DIM);
  pc.lo = rd.vec<double>(MAX_DIM);
  pc.hi = rd.vec<double>(MAX_DIM);
  pc.dre = rd.vec<double>(big);
  pc.dim = rd.vec<double>(big);
  pc.psd = rd.vec<double>(big);
  pc.geom = rd.vec<double>(9 * MAX_DET);
  pc.fid = rd.vec<double>(MAX_DIM);
  pc.mu = rd.vec<double>(MAX_DIM);
  pc.per = rd.vec<int>(MAX_DIM);
  const DevState st = rd.val<DevState>();
  auto u = rd.vec<double>(big), lam = rd.vec<double>(big), du = rd.vec<double>(big), dlam = rd.vec<double>(big),
       dlogx = rd.vec<double>(big), dlogw = rd.vec<double>(big);
  auto diter = rd.vec<int>(big), dslot = rd.vec<int>(big), dnlive = rd.vec<int>(big);
  auto trace = rd.vec<IterRec>(big);
  if (!rd.ok || rd.n != size) return fail(NS_E_ARG, "malformed checkpoint");
  ns_problem P{};
  P.model = ps.model; P.likelihood = ps.likelihood; P.n_dim = ps.n_dim; P.n_bins = ps.n_bins; P.n_det = ps.n_det;
  P.rb_n_bins = ps.rb_n_bins; P.f_lo = ps.f_lo; P.df = ps.df; P.gmst = ps.gmst;
  P.fixed_dist_mpc = ps.fixed_dist_mpc; P.gauss_sigma = ps.gauss_sigma;
  const size_t nd = (size_t)std::max(ps.n_dim, 0);
  const size_t nbd = ps.likelihood == NS_LIKE_GAUSS ? 0 : (size_t)std::max(ps.n_det, 0) * std::max(ps.n_bins, 0);
  if (pc.kind.size() != nd || pc.lo.size() != nd || pc.hi.size() != nd || pc.dre.size() != nbd ||
      pc.dim.size() != nbd || pc.psd.size() != nbd)
    return fail(NS_E_ARG, "checkpoint arrays do not match the problem sizes");
  P.prior_kind = pc.kind.data(); P.prior_lo = pc.lo.data(); P.prior_hi = pc.hi.data();
  P.data_re = nbd ? pc.dre.data() : nullptr;
  P.data_im = nbd ? pc.dim.data() : nullptr;
  P.psd = nbd ? pc.psd.data() : nullptr;
  P.det_geom = pc.geom.empty() ? nullptr : pc.geom.data();
  P.rb_fiducial = pc.fid.empty() ? nullptr : pc.fid.data();
  P.gauss_mu = pc.mu.empty() ? nullptr : pc.mu.data();
  P.periodic = pc.per.empty() ? nullptr : pc.per.data();
  if (!pc.per.empty() && pc.per.size() != nd) return fail(NS_E_ARG, "checkpoint periodic mask size");
  if (P.det_geom && pc.geom.size() != 9 * (size_t)P.n_det) return fail(NS_E_ARG, "checkpoint detector geometry size");
  if (P.rb_fiducial && pc.fid.size() != nd) return fail(NS_E_ARG, "checkpoint fiducial size");
  if (P.gauss_mu && pc.mu.size() != nd) return fail(NS_E_ARG, "checkpoint Gaussian mean size");
  const size_t n = (size_t)std::max(O.n_live, 0), d = nd;
  const long long ndead = st.n_dead;
  if (ndead < 0 || u.size() != n * d || lam.size() != n || du.size() != (size_t)ndead * d ||
      dlam.size() != (size_t)ndead || dlogx.size() != (size_t)ndead || dlogw.size() != (size_t)ndead ||
      diter.size() != (size_t)ndead || dslot.size() != (size_t)ndead || dnlive.size() != (size_t)ndead ||
      ndead > (long long)O.max_iter * O.n_delete ||
      (long long)trace.size() != std::min<long long>(std::max(st.iter, 0), std::max(O.max_iter, 0)))
    return fail(NS_E_ARG, "checkpoint state does not match the run sizes");
  ns_run* r = nullptr;
  int rc = run_create(&r, &P, &O, static_cast<hipStream_t>(stream), packed != 0);
  if (rc) return rc;
  const RunDev& R = r->R;
  *r->h_state = st;
  hipError_t e = hipMemcpyAsync(R.state, r->h_state, sizeof(DevState), hipMemcpyHostToDevice, r->st);
  if (e == hipSuccess) e = hipMemcpyAsync(R.u, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice, r->st);
  if (e == hipSuccess) e = hipMemcpyAsync(R.lam, lam.data(), n * sizeof(double), hipMemcpyHostToDevice, r->st);
  if (e == hipSuccess && ndead) {
    e = hipMemcpyAsync(R.du, du.data(), du.size() * sizeof(double), hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess) e = hipMemcpyAsync(R.dlam, dlam.data(), ndead * sizeof(double), hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess) e = hipMemcpyAsync(R.dlogx, dlogx.data(), ndead * sizeof(double), hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess) e = hipMemcpyAsync(R.dlogw, dlogw.data(), ndead * sizeof(double), hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess) e = hipMemcpyAsync(R.diter, diter.data(), ndead * sizeof(int), hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess) e = hipMemcpyAsync(R.dslot, dslot.data(), ndead * sizeof(int), hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess) e = hipMemcpyAsync(R.dnlive, dnlive.data(), ndead * sizeof(int), hipMemcpyHostToDevice, r->st);
  }
  if (e == hipSuccess && !trace.empty())
    e = hipMemcpyAsync(R.trace, trace.data(), trace.size() * sizeof(IterRec), hipMemcpyHostToDevice, r->st);
  if (e == hipSuccess) e = hipStreamSynchronize(r->st);
  if (e != hipSuccess) {
    ns_free(r);
    return fail(NS_E_HIP, "restoring the checkpoint: %s", hipGetErrorString(e));
  }
  *out = r;
  return NS_OK;
}

void ns_free(ns_run* r) {
  if (!r) return;
  (void)hipStreamSynchronize(r->st);
  delete r;
}

}  // extern "C"
