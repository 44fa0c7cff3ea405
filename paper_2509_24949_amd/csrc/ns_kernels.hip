// Kernels of libns for gfx950 (wave64).
//
//  * k_rank       bit-exact selection: the rank of every live point in the
//                 total order (order key, slot); the k lowest die.
//  * k_prep       one workgroup: evidence and prior-volume update of the k
//                 deaths, dead-point record, covariance of the live points
//                 and its Cholesky factor, survivor list, chain start points.
//  * k_slice      one workgroup per chain: the whole constrained slice walk
//                 of the iteration with the chain state in registers and the
//                 likelihood tables in LDS.  The per-probe source setup
//                 (masses, amplitude, antenna patterns, PN coefficients) is
//                 computed lane-parallel for a batch of candidate probes
//                 whose positions are known in advance (the step-out points
//                 and the shrink candidates), then each probe's bins are
//                 spread over the workgroup and reduced once.
//  * k_term       one workgroup: live evidence, termination flag, counters.
//  * k_loglike    batched fused likelihood: each wavefront sets up 64 probes
//                 (one per lane) and then evaluates them one after another
//                 with all 64 lanes over the frequency bins.
#include <float.h>
#include <math.h>

#include "ns_internal.h"

namespace ns {

namespace {

constexpr double NEG_INF = -__builtin_inf();

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ inline long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Value of lane `src` of this wavefront (src uniform), as a scalar.
__device__ inline double lane_d(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

__device__ inline int lane_i(int v, int src) { return __builtin_amdgcn_readlane(v, src); }

// Block-wide reductions for NT-thread workgroups; every thread receives the
// result, combined in a fixed order.
template <int NT>
__device__ inline double block_sum(double v, double* sbuf) {
  constexpr int NW = NT / 64;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sbuf[wv] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) t += sbuf[w];
  return t;
}

template <int NT>
__device__ inline double block_max(double v, double* sbuf) {
  constexpr int NW = NT / 64;
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sbuf[wv] = v;
  __syncthreads();
  double t = NEG_INF;
#pragma unroll
  for (int w = 0; w < NW; ++w) t = fmax(t, sbuf[w]);
  return t;
}

// Inclusive Hillis-Steele scan over NT values held one per thread.
template <int NT, typename T>
__device__ inline T block_inclusive_scan(T v, T* sbuf) {
  __syncthreads();
  sbuf[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < NT; o <<= 1) {
    T add = (threadIdx.x >= (unsigned)o) ? sbuf[threadIdx.x - o] : T(0);
    __syncthreads();
    v += add;
    sbuf[threadIdx.x] = v;
    __syncthreads();
  }
  return v;
}

// ---------------------------------------------------------------- tables
// Pointers of the full-grid tables as one chain or probe sees them: either
// the HBM arrays or a copy of their active prefix in LDS.
struct TabView {
  const double* f;
  const double* f13;
  const double* lnf3;
  const double* fm53;
  const double2* dw;
  int dstride;
};

template <int NDET>
__device__ inline TabView stage_tables(const ModelDev& M, const Tables& T, bool use_lds, double* lds, int tid,
                                       int nt) {
  TabView V;
  if (!use_lds) {
    V.f = T.f; V.f13 = T.f13; V.lnf3 = T.lnf3; V.fm53 = T.fm53; V.dw = T.dw; V.dstride = M.n_bins;
    return V;
  }
  const int K = M.k_lim;
  double* f = lds;
  double* f13 = f + K;
  double* lnf3 = f13 + K;
  double* fm53 = lnf3 + K;
  double2* dw = reinterpret_cast<double2*>(fm53 + K);
  for (int k = tid; k < K; k += nt) {
    f[k] = T.f[k];
    f13[k] = T.f13[k];
    lnf3[k] = T.lnf3[k];
    fm53[k] = T.fm53[k];
#pragma unroll
    for (int d = 0; d < NDET; ++d) dw[d * K + k] = T.dw[(size_t)d * M.n_bins + k];
  }
  V.f = f; V.f13 = f13; V.lnf3 = lnf3; V.fm53 = fm53; V.dw = dw; V.dstride = K;
  return V;
}

// The coefficients of the probe held by lane `src`, broadcast to the wave.
template <int NDET>
__device__ inline Probe probe_from_lane(const Probe& p, int src) {
  Probe b;
  b.x = lane_d(p.x, src);
  b.lnx = lane_d(p.lnx, src);
  b.pref = lane_d(p.pref, src);
  b.c2 = lane_d(p.c2, src);
  b.c3 = lane_d(p.c3, src);
  b.c4 = lane_d(p.c4, src);
  b.c5 = lane_d(p.c5, src);
  b.c5l = lane_d(p.c5l, src);
  b.c6 = lane_d(p.c6, src);
  b.c6l = lane_d(p.c6l, src);
  b.c7 = lane_d(p.c7, src);
  b.tc = lane_d(p.tc, src);
  b.ph0 = lane_d(p.ph0, src);
#pragma unroll
  for (int d = 0; d < NDET; ++d) {
    b.kre[d] = lane_d(p.kre[d], src);
    b.kim[d] = lane_d(p.kim[d], src);
    b.dt[d] = lane_d(p.dt[d], src);
  }
  b.hh = lane_d(p.hh, src);
  b.f_isco = 0.0;
  b.k_act = lane_i(p.k_act, src);
  return b;
}

// This thread's share of <d|h> summed over detectors, for the active bins
// k = lane, lane + nl, ...:  sum_d Re[A K_d sum_k conj(Dw_dk) e^{-i Phi_dk}].
// Per detector the bin sums a_d = sum (Dr c - Di s) and b_d = sum (Dr s + Di c)
// are folded with A K_d = (kre, kim) as kre a_d + kim b_d before returning, so a
// probe needs a single reduction.
template <int NDET>
__device__ inline double fullgrid_partial(const Probe& p, const TabView& V, int lane, int nl) {
  double a[NDET], b[NDET];
#pragma unroll
  for (int d = 0; d < NDET; ++d) { a[d] = 0.0; b[d] = 0.0; }
  for (int k = lane; k < p.k_act; k += nl) {
    const double f = V.f[k];
    const double psi = phase_cycles(p, f, V.f13[k], V.lnf3[k], V.fm53[k]);
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
      double sn, cs;
      sincos_cycles(fma(f, p.dt[d], psi), &sn, &cs);
      const double2 D = V.dw[d * V.dstride + k];
      a[d] = fma(D.x, cs, fma(-D.y, sn, a[d]));
      b[d] = fma(D.x, sn, fma(D.y, cs, b[d]));
    }
  }
  double part = 0.0;
#pragma unroll
  for (int d = 0; d < NDET; ++d) part = fma(p.kre[d], a[d], fma(p.kim[d], b[d], part));
  return part;
}

__device__ inline double gauss_lambda(const ModelDev& M, const double* u) {
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < MAX_DIM; ++i)
    if (i < M.n_dim) {
      double z = u[i] - M.gauss_mu[i];
      acc = fma(-z * z, M.gauss_inv2s2, acc);
    }
  return acc + M.gauss_norm;
}

// ------------------------------------------------------------ build tables
__global__ void k_build_tables(const ModelDev* __restrict__ Mp, const double* dre, const double* dim,
                               const double* psd, double* f, double* f13, double* lnf3, double* fm53, double2* dw,
                               double* hw) {
  const ModelDev& M = *Mp;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M.n_bins) return;
  const double fk = fma((double)k, M.df, M.f_lo);
  const double lf = log(fk);
  f[k] = fk;
  f13[k] = cbrt(fk);
  lnf3[k] = lf / 3.0;
  fm53[k] = exp(-5.0 / 3.0 * lf);
  const double a = 4.0 * M.df * exp(-7.0 / 6.0 * lf);
  const double b = 4.0 * M.df * exp(-7.0 / 3.0 * lf);
  for (int d = 0; d < M.n_det; ++d) {
    const size_t o = (size_t)d * M.n_bins + k;
    const double s = psd[o];
    dw[o] = make_double2(a * dre[o] / s, a * dim[o] / s);
    hw[o] = b / s;
  }
}

// Inclusive prefix sums of rows of length n (one workgroup per row).
__global__ __launch_bounds__(1024) void k_prefix_rows(const double* in, double* out, int n) {
  __shared__ double sbuf[1024];
  const double* x = in + (size_t)blockIdx.x * n;
  double* y = out + (size_t)blockIdx.x * n;
  const int C = (n + 1023) / 1024;
  const int b = threadIdx.x * C, e = min(n, b + C);
  double s = 0.0;
  for (int i = b; i < e; ++i) s += x[i];
  double incl = block_inclusive_scan<1024, double>(s, sbuf);
  double run = incl - s;
  for (int i = b; i < e; ++i) {
    run += x[i];
    y[i] = run;
  }
}

// ---------------------------------------------------------------- init
__global__ void k_init_live(int n, int d, uint64_t k0, uint64_t k1, double* u) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int i = 0; i < d; i += 4) {
    u64x4 b = philox(0, (uint64_t)j, 0, purpose_word(P_INIT, (uint64_t)(i >> 2)), k0, k1);
    for (int q = 0; q < 4 && i + q < d; ++q) u[(size_t)j * d + i + q] = unif53(b.x[q]);
  }
}

// ---------------------------------------------------------- batched lambda
// Each wavefront takes 64 consecutive probes: lane l sets up probe base + l,
// then the wave evaluates the probes one at a time over the bins.
template <int NDET, int LK, bool LDS>
__global__ __launch_bounds__(256) void k_loglike(const ModelDev* __restrict__ Mp, Tables T, RBTables RB,
                                                 const double* __restrict__ u, long n, double* __restrict__ out) {
  extern __shared__ double smem[];
  const ModelDev& M = *Mp;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  TabView V{};
  if (LK == LK_FULL) {
    V = stage_tables<NDET>(M, T, LDS, smem, tid, 256);
    if (LDS) __syncthreads();
  }
  const int d = M.n_dim;
  for (long base = ((long)blockIdx.x * 4 + wv) * 64; base < n; base += (long)gridDim.x * 256) {
    const long i = base + lane;
    const long src = i < n ? i : base;
    double y[MAX_DIM];
#pragma unroll
    for (int q = 0; q < MAX_DIM; ++q) y[q] = (q < d) ? u[src * d + q] : 0.0;
    double mine;
    if (LK == LK_GAUSS) {
      mine = gauss_lambda(M, y);
    } else {
      Probe pr;
      make_probe(M, T.hpre, y, &pr);
      mine = 0.0;
      const int cnt = (n - base) < 64 ? (int)(n - base) : 64;
      for (int p = 0; p < cnt; ++p) {
        const Probe pb = probe_from_lane<NDET>(pr, p);
        const double tot = wave_sum(fullgrid_partial<NDET>(pb, V, lane, 64));
        if (lane == p) mine = tot - 0.5 * pb.hh;
      }
    }
    if (i < n) out[i] = mine;
  }
}

// ---------------------------------------------------------------- select
__global__ __launch_bounds__(256) void k_rank(const double* __restrict__ lam, int n, int k, int* rank, int* dead,
                                              double* lstar, const int* done) {
  if (done && *done) return;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= n) return;
  const uint64_t ki = order_key(lam[i]);
  int cnt = 0;
  for (int j = lane; j < n; j += 64) {
    const uint64_t kj = order_key(lam[j]);
    cnt += (kj < ki) || (kj == ki && j < i);
  }
  cnt = (int)wave_sum_ll(cnt);
  if (lane == 0) {
    if (rank) rank[i] = cnt;
    if (cnt < k) dead[cnt] = i;
    if (cnt == k - 1 && lstar) *lstar = order_value(lam[i]);
  }
}

// ------------------------------------------------------------- iteration prep
// One workgroup of 1024 threads.  Dynamic LDS: n ints (survivor list).
__global__ __launch_bounds__(1024) void k_prep(RunDev R) {
  extern __shared__ int s_surv[];
  __shared__ double sbuf[1024];
  __shared__ double smean[MAX_DIM];
  __shared__ double scov[MAX_DIM * MAX_DIM];
  __shared__ int sint[1024];
  DevState* S = R.state;
  const int done0 = S->done;
  if (done0) return;
  const int n = R.n, k = R.k, d = R.d, tid = threadIdx.x;
  const long long nd0 = S->n_dead;
  const double logX0 = S->logX, logZ0 = S->logZ, H0 = S->H;
  const int it = S->iter;
  __syncthreads();
  if (nd0 + k > R.cap) {
    if (tid == 0) S->done = 2;
    return;
  }

  // ---- evidence: the j-th death shrinks log X by 1/(n-j); its weight is the
  // shell between consecutive volumes, X_{j-1} (1 - e^{-1/(n-j)}).
  const int C = (k + 1023) / 1024;
  const int jb = tid * C, je = min(k, jb + C);
  double csum = 0.0;
  for (int j = jb; j < je; ++j) csum += 1.0 / (double)(n - j);
  double incl = block_inclusive_scan<1024, double>(csum, sbuf);
  double lx = logX0 - (incl - csum);
  double mloc = NEG_INF;
  for (int j = jb; j < je; ++j) {
    const int slot = R.dead[j];
    const double lraw = R.lam[slot];
    const double l = order_value(lraw);
    const double inv = 1.0 / (double)(n - j);
    const double lw = l + lx + log(-expm1(-inv));
    const double lxn = lx - inv;
    const long long q = nd0 + j;
    for (int i = 0; i < d; ++i) R.du[q * d + i] = R.u[(size_t)slot * d + i];
    R.dlam[q] = lraw;
    R.dlogx[q] = lxn;
    R.dlogw[q] = lw;
    R.diter[q] = it;
    R.dslot[q] = slot;
    R.dnlive[q] = n - j;
    mloc = fmax(mloc, lw);
    lx = lxn;
  }
  const double total = block_sum<1024>(csum, sbuf);   // sum of 1/(n-j) over the batch
  double m = block_max<1024>(mloc, sbuf);
  m = fmax(m, logZ0);
  double s1 = 0.0, s2 = 0.0;
  if (m > NEG_INF) {
    for (int j = jb; j < je; ++j) {
      const double lw = R.dlogw[nd0 + j];
      if (lw > NEG_INF) {
        const double e = exp(lw - m);
        s1 += e;
        s2 += e * order_value(R.dlam[nd0 + j]);
      }
    }
  }
  s1 = block_sum<1024>(s1, sbuf);
  s2 = block_sum<1024>(s2, sbuf);
  if (tid == 0) {
    double logZ1 = logZ0, H1 = H0;
    if (m > NEG_INF) {
      const double zold = (logZ0 > NEG_INF) ? exp(logZ0 - m) : 0.0;
      logZ1 = m + log(zold + s1);
      H1 = s2 * exp(m - logZ1) - logZ1;
      if (logZ0 > NEG_INF) H1 += exp(logZ0 - logZ1) * (H0 + logZ0);
    }
    S->logX = logX0 - total;
    S->logZ = logZ1;
    S->H = H1;
    S->lstar = order_value(R.lam[R.dead[k - 1]]);
    S->n_dead = nd0 + k;
  }

  // ---- covariance of all n live points (before removal), 1/(n-1)
  double part[MAX_DIM];
#pragma unroll
  for (int i = 0; i < MAX_DIM; ++i) part[i] = 0.0;
  for (int j = tid; j < n; j += 1024) {
#pragma unroll
    for (int i = 0; i < MAX_DIM; ++i)
      if (i < d) part[i] += R.u[(size_t)j * d + i];
  }
#pragma unroll
  for (int i = 0; i < MAX_DIM; ++i) {
    if (i < d) {
      const double t = block_sum<1024>(part[i], sbuf);
      if (tid == 0) smean[i] = t / n;
    }
  }
  __syncthreads();
  const int E = d * (d + 1) / 2;
  const int G = 1024 / E;
  const int e = tid % E, g = tid / E;
  int ea = 0, eb = 0;
  {
    int r = e;
    while (r > ea) { r -= ea + 1; ++ea; }   // e -> (a, b) with a >= b, row-major lower triangle
    eb = r;
  }
  double cs = 0.0;
  if (g < G)
    for (int j = g; j < n; j += G)
      cs += (R.u[(size_t)j * d + ea] - smean[ea]) * (R.u[(size_t)j * d + eb] - smean[eb]);
  __syncthreads();
  sbuf[tid] = cs;
  __syncthreads();
  if (tid < E) {
    double t = 0.0;
    for (int gg = 0; gg < G; ++gg) t += sbuf[tid + gg * E];
    t /= (double)(n - 1);
    scov[ea * d + eb] = t;
    scov[eb * d + ea] = t;
  }
  __syncthreads();
  if (tid == 0) {
    // Cholesky factor; on failure add 1e-12 tr/d to the diagonal and retry
    double L[MAX_DIM * MAX_DIM];
    bool ok = false;
    for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
      if (attempt == 1) {
        double tr = 0.0;
        for (int i = 0; i < d; ++i) tr += scov[i * d + i];
        for (int i = 0; i < d; ++i) scov[i * d + i] += 1e-12 * tr / d;
      }
      ok = true;
      for (int i = 0; i < d && ok; ++i)
        for (int j = 0; j <= i; ++j) {
          double s = scov[i * d + j];
          for (int q = 0; q < j; ++q) s -= L[i * d + q] * L[j * d + q];
          if (i == j) {
            if (!(s > 0.0)) { ok = false; break; }
            L[i * d + i] = sqrt(s);
          } else {
            L[i * d + j] = s / L[j * d + j];
          }
        }
    }
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) R.chol[i * d + j] = ok ? (j <= i ? L[i * d + j] : 0.0) : (i == j ? 1e-6 : 0.0);
  }

  // ---- survivors in ascending slot order, then the chain start points
  const int C2 = (n + 1023) / 1024;
  const int ib = tid * C2, ie = min(n, ib + C2);
  int cnt = 0;
  for (int i = ib; i < ie; ++i) cnt += (R.rank[i] >= k);
  int icl = block_inclusive_scan<1024, int>(cnt, sint);
  int pos = icl - cnt;
  for (int i = ib; i < ie; ++i)
    if (R.rank[i] >= k) s_surv[pos++] = i;
  __syncthreads();
  const int ns = n - k;
  for (int j = tid; j < k; j += 1024) {
    u64x4 b = philox((uint64_t)it, (uint64_t)j, 0, purpose_word(P_PICK, 0), R.key0, R.key1);
    const int idx = (int)floor(unif53(b.x[0]) * (double)ns);
    R.start[j] = s_surv[idx < ns ? idx : ns - 1];
  }
}

// ------------------------------------------------------------ slice chains
// One workgroup of NT threads runs chain j = blockIdx.x for all n_steps
// steps.  State, direction and bracket are uniform across the workgroup and
// every wavefront computes the same candidate batches, so probe coefficients
// are broadcast within a wave with readlane.  A probe's bins are spread over
// all NT threads; one value is reduced per probe.
template <int NDET, int NT, int LK, bool LDS>
__global__ __launch_bounds__(NT) void k_slice(const ModelDev* __restrict__ Mp, Tables T, RBTables RB, RunDev R) {
  constexpr int NW = NT / 64;
  constexpr int SOB = 32;          // step-out candidates per side and batch
  constexpr int SHB = 8;           // shrink candidates per batch
  extern __shared__ double smem[];
  const ModelDev& M = *Mp;
  DevState* S = R.state;
  if (S->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int j = blockIdx.x;
  const int d = R.d;
  const uint64_t t = (uint64_t)S->iter;
  const double lstar = S->lstar;
  double* sL = smem;                         // [MAX_DIM * MAX_DIM]
  double* sred = sL + MAX_DIM * MAX_DIM;     // [2][NW]
  double* stab = sred + 2 * 8;
  for (int i = tid; i < d * d; i += NT) sL[i] = R.chol[i];
  TabView V{};
  if (LK == LK_FULL) V = stage_tables<NDET>(M, T, LDS, stab, tid, NT);
  __syncthreads();

  int buf = 0;
  int nprobe = 0;
  long long nbins = 0;
  // this lane's candidate of the current batch
  Probe pr;
  double glam = 0.0;            // Gaussian test likelihood of the candidate
  bool cin = false;             // candidate inside the unit cube

  auto setup = [&](double tt, const double* x, const double* dir) {
    double y[MAX_DIM];
    cin = true;
#pragma unroll
    for (int i = 0; i < MAX_DIM; ++i) {
      y[i] = (i < d) ? fma(tt, dir[i], x[i]) : 0.0;
      if (i < d && !(y[i] >= 0.0 && y[i] <= 1.0)) cin = false;
    }
    if (!cin) {
#pragma unroll
      for (int i = 0; i < MAX_DIM; ++i) y[i] = 0.5;   // a harmless point; never evaluated
    }
    if (LK == LK_GAUSS) glam = gauss_lambda(M, y);
    else make_probe(M, T.hpre, y, &pr);
  };
  // lambda of the candidate held by lane src of every wavefront
  auto eval = [&](int src) -> double {
    ++nprobe;
    if (LK == LK_GAUSS) return lane_d(glam, src);
    const Probe pb = probe_from_lane<NDET>(pr, src);
    nbins += pb.k_act;
    double tot = wave_sum(fullgrid_partial<NDET>(pb, V, tid, NT));
    if constexpr (NW > 1) {
      double* rb = sred + buf * NW;
      if (lane == 0) rb[wv] = tot;
      __syncthreads();
      tot = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) tot += rb[w];
      buf ^= 1;
    }
    return tot - 0.5 * pb.hh;
  };

  const int start = R.start[j];
  double x[MAX_DIM];
#pragma unroll
  for (int i = 0; i < MAX_DIM; ++i) x[i] = (i < d) ? R.u[(size_t)start * d + i] : 0.0;
  double lx = R.lam[start];
  const int nbd = (d + 3) >> 2;      // DIR blocks
  const double w = R.width;

  for (int s = 0; s < R.m; ++s) {
    // lanes 0..nbd-1: direction blocks (two Box-Muller pairs each); lane nbd:
    // the width block; lanes nbd+1, nbd+2: the first eight shrink uniforms
    double r0 = 0, r1 = 0, r2 = 0, r3 = 0;
    if (lane < nbd + 3) {
      uint64_t pw;
      if (lane < nbd) pw = purpose_word(P_DIR, (uint64_t)lane);
      else if (lane == nbd) pw = purpose_word(P_WIDTH, 0);
      else pw = purpose_word(P_SHRINK, (uint64_t)(lane - nbd - 1));
      u64x4 b = philox(t, (uint64_t)j, (uint64_t)s, pw, R.key0, R.key1);
      r0 = unif53(b.x[0]); r1 = unif53(b.x[1]); r2 = unif53(b.x[2]); r3 = unif53(b.x[3]);
      if (lane < nbd) {
        double sa, ca, sb, cb;
        const double ra = sqrt(-2.0 * log(1.0 - r0));
        sincos_cycles(r1, &sa, &ca);
        const double rb = sqrt(-2.0 * log(1.0 - r2));
        sincos_cycles(r3, &sb, &cb);
        r0 = ra * ca; r1 = ra * sa; r2 = rb * cb; r3 = rb * sb;
      }
    }
    double z[MAX_DIM];
#pragma unroll
    for (int i = 0; i < MAX_DIM; ++i) {
      const double v = ((i & 3) == 0) ? r0 : ((i & 3) == 1) ? r1 : ((i & 3) == 2) ? r2 : r3;
      z[i] = (i < d) ? lane_d(v, i >> 2) : 0.0;
    }
    const double uw = lane_d(r0, nbd), uj = lane_d(r1, nbd);
    // direction L z / |z|
    double nrm = 0.0;
#pragma unroll
    for (int i = 0; i < MAX_DIM; ++i)
      if (i < d) nrm += z[i] * z[i];
    nrm = sqrt(nrm);
    double dir[MAX_DIM];
#pragma unroll
    for (int a = 0; a < MAX_DIM; ++a) {
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < MAX_DIM; ++b)
        if (b <= a && a < d) acc += sL[a * d + b] * z[b];
      dir[a] = acc / nrm;
    }

    // ---- step out.  Candidate positions are fixed before any is evaluated:
    // lane l < 32 holds the left point after l successful steps, lane 32 + l
    // the right one, so the sequential walk only reads results.
    double lo = -w * uw, hi = lo + w;
    int J = (int)floor(R.max_stepout * uj);
    int K = R.max_stepout - 1 - J;
    for (int jl = 0, jh = 0; J > 0 || K > 0;) {
      {
        const bool left = lane < SOB;
        const int steps = left ? jl + lane : jh + lane - SOB;   // further steps beyond the current end
        double tt = left ? lo : hi;
        for (int q = (left ? jl : jh); q < steps; ++q) tt = left ? tt - w : tt + w;
        setup(tt, x, dir);
      }
      const unsigned long long inb = __ballot(cin);
      int q = 0;
      while (J > 0 && q < SOB) {
        if (!((inb >> q) & 1ull)) { J = 0; break; }
        if (!(eval(q) > lstar)) { J = 0; break; }
        lo -= w;
        --J;
        ++q;
      }
      jl += q;
      q = 0;
      while (K > 0 && q < SOB) {
        if (!((inb >> (SOB + q)) & 1ull)) { K = 0; break; }
        if (!(eval(SOB + q) > lstar)) { K = 0; break; }
        hi += w;
        --K;
        ++q;
      }
      jh += q;
    }

    // ---- shrink.  Under the hypothesis that every earlier candidate was
    // rejected the candidate sequence is fixed, so batches of SHB candidates
    // are set up together; the first accepted one ends the step.
    for (int a0 = 0; a0 < R.max_shrink; a0 += SHB) {
      double tl = 0.0;          // candidate of lane a - a0
      {
        double l2 = lo, h2 = hi;
        for (int q = 0; q < SHB; ++q) {
          const int a = a0 + q;
          double ua;
          if (a < 8) {
            const double v0 = ((a & 3) == 0) ? r0 : ((a & 3) == 1) ? r1 : ((a & 3) == 2) ? r2 : r3;
            ua = lane_d(v0, nbd + 1 + (a >> 2));
          } else {
            u64x4 b = philox(t, (uint64_t)j, (uint64_t)s, purpose_word(P_SHRINK, (uint64_t)(a >> 2)), R.key0,
                             R.key1);
            ua = unif53(b.x[a & 3]);
          }
          const double tt = fma(ua, h2 - l2, l2);
          if (lane == q) tl = tt;
          if (tt < 0.0) l2 = tt; else h2 = tt;
        }
      }
      setup(tl, x, dir);
      const unsigned long long inb = __ballot(cin);
      bool accepted = false;
      for (int q = 0; q < SHB && a0 + q < R.max_shrink; ++q) {
        const double tt = lane_d(tl, q);
        if ((inb >> q) & 1ull) {
          const double ly = eval(q);
          if (ly > lstar) {
#pragma unroll
            for (int i = 0; i < MAX_DIM; ++i) x[i] = (i < d) ? fma(tt, dir[i], x[i]) : 0.0;
            lx = ly;
            accepted = true;
            break;
          }
        }
        if (tt < 0.0) lo = tt; else hi = tt;
      }
      if (accepted) break;
    }
  }
  if (tid == 0) {
    const int slot = R.dead[j];
    for (int i = 0; i < d; ++i) R.u[(size_t)slot * d + i] = x[i];
    R.lam[slot] = lx;
    R.probes[j] = nprobe;
    R.bins[j] = nbins;
  }
}

// ------------------------------------------------------------- termination
__global__ __launch_bounds__(1024) void k_term(RunDev R) {
  __shared__ double sbuf[1024];
  DevState* S = R.state;
  if (S->done) return;
  const int n = R.n, tid = threadIdx.x;
  double m = NEG_INF;
  for (int i = tid; i < n; i += 1024) m = fmax(m, order_value(R.lam[i]));
  m = block_max<1024>(m, sbuf);
  double s = 0.0;
  for (int i = tid; i < n; i += 1024) s += exp(order_value(R.lam[i]) - m);
  s = block_sum<1024>(s, sbuf);
  double pe = 0.0, pb = 0.0;
  for (int j = tid; j < R.k; j += 1024) {
    pe += (double)R.probes[j];
    pb += (double)R.bins[j];
  }
  pe = block_sum<1024>(pe, sbuf);
  pb = block_sum<1024>(pb, sbuf);
  if (tid == 0) {
    const double logz_live = S->logX + m + log(s / n);
    int done = 0;
    if (R.log_term > NEG_INF && logz_live - S->logZ < R.log_term) done = 1;
    if (S->n_dead + R.k > R.cap) done = 2;
    S->n_evals += (long long)pe;
    S->n_bin_terms += (long long)pb;
    S->iter += 1;
    S->done = done;
  }
}

// ---------------------------------------------------------------- waveform
__global__ void k_waveform(const ModelDev* __restrict__ Mp, const double* theta, int det, int apply_cut, double* hre,
                           double* him) {
  const ModelDev& M = *Mp;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M.n_bins) return;
  Phys s;
  phys_from_theta(M, theta, &s);
  Probe p;
  probe_from_phys(M, s, nullptr, &p);
  const double f = fma((double)k, M.df, M.f_lo);
  if (apply_cut && k >= p.k_act) {
    hre[k] = 0.0;
    him[k] = 0.0;
    return;
  }
  const double lf = log(f);
  const double psi = phase_cycles(p, f, cbrt(f), lf / 3.0, exp(-5.0 / 3.0 * lf));
  double sn, cs;
  sincos_cycles(fma(f, p.dt[det], psi), &sn, &cs);
  const double a = exp(-7.0 / 6.0 * lf);
  // h = A K f^(-7/6) e^{-i Phi}
  hre[k] = a * (p.kre[det] * cs + p.kim[det] * sn);
  him[k] = a * (p.kim[det] * cs - p.kre[det] * sn);
}

// ------------------------------------------------------------- finalisation
// Block 0: the final evidence (each live point takes X_end / n), the
// information H and the Kish effective sample size.  Block r >= 1: replica
// r-1 of log Z with every log-shrinkage redrawn, log t = log U / n_j.
// out: [0] log Z, [1] H, [2] ESS, [3 + r] replica log Z.
__global__ __launch_bounds__(1024) void k_final(RunDev R, int n_sim, double* out) {
  __shared__ double sbuf[1024];
  const DevState* S = R.state;
  const long long nd = S->n_dead;
  const int n = R.n, tid = threadIdx.x;
  const double logn = log((double)n);
  double m = NEG_INF;
  for (int i = tid; i < n; i += 1024) m = fmax(m, order_value(R.lam[i]));
  m = block_max<1024>(m, sbuf);
  if (blockIdx.x == 0) {
    double s = 0.0;
    if (m > NEG_INF)
      for (int i = tid; i < n; i += 1024) s += exp(order_value(R.lam[i]) - m);
    s = block_sum<1024>(s, sbuf);
    const double zl = (m > NEG_INF) ? S->logX + m + log(s) - logn : NEG_INF;
    double logZ = S->logZ;
    if (zl > NEG_INF) logZ = (logZ > NEG_INF) ? fmax(logZ, zl) + log1p(exp(-fabs(logZ - zl))) : zl;
    double h = 0.0, p2 = 0.0;
    for (long long q = tid; q < nd; q += 1024) {
      const double lw = R.dlogw[q];
      if (lw > NEG_INF) {
        const double pq = exp(lw - logZ);
        h += pq * order_value(R.dlam[q]);
        p2 += pq * pq;
      }
    }
    for (int i = tid; i < n; i += 1024) {
      const double l = order_value(R.lam[i]);
      if (l > NEG_INF) {
        const double pq = exp(l + S->logX - logn - logZ);
        h += pq * l;
        p2 += pq * pq;
      }
    }
    h = block_sum<1024>(h, sbuf);
    p2 = block_sum<1024>(p2, sbuf);
    if (tid == 0) {
      out[0] = logZ;
      out[1] = h - logZ;
      out[2] = 1.0 / p2;
    }
    return;
  }
  const uint64_t rep = (uint64_t)(blockIdx.x - 1);
  const long long C = (nd + 1023) / 1024;
  const long long qb = (long long)tid * C, qe = (qb + C < nd) ? qb + C : nd;
  auto logt = [&](long long q) {
    u64x4 b = philox(rep, (uint64_t)q, 0, purpose_word(P_SIGMA, 0), R.key0, R.key1);
    return log(1.0 - unif53(b.x[0])) / (double)R.dnlive[q];
  };
  double cs = 0.0;
  for (long long q = qb; q < qe; ++q) cs += logt(q);
  __shared__ double sscan[1024];
  const double incl = block_inclusive_scan<1024, double>(cs, sscan);
  double lx = incl - cs;
  double mloc = NEG_INF;
  for (long long q = qb; q < qe; ++q) {
    const double lt = logt(q);
    const double lw = order_value(R.dlam[q]) + lx + log(-expm1(lt));
    mloc = fmax(mloc, lw);
    lx += lt;
  }
  const double lxend = block_sum<1024>(cs, sbuf);
  double mm = block_max<1024>(mloc, sbuf);
  const double live_top = (m > NEG_INF) ? m + lxend - logn : NEG_INF;
  mm = fmax(mm, live_top);
  double s = 0.0;
  lx = incl - cs;
  for (long long q = qb; q < qe; ++q) {
    const double lt = logt(q);
    const double lw = order_value(R.dlam[q]) + lx + log(-expm1(lt));
    if (lw > NEG_INF) s += exp(lw - mm);
    lx += lt;
  }
  for (int i = tid; i < n; i += 1024) {
    const double l = order_value(R.lam[i]);
    if (l > NEG_INF) s += exp(l + lxend - logn - mm);
  }
  s = block_sum<1024>(s, sbuf);
  if (tid == 0) out[3 + rep] = mm + log(s);
}

// Weighted samples: dead points then live points, physical parameters and
// log-weights normalised by the final log Z.
__global__ void k_samples(const ModelDev* __restrict__ Mp, RunDev R, double logZ, double* theta, double* logl,
                          double* logw) {
  const ModelDev& M = *Mp;
  const long long nd = R.state->n_dead;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nd + R.n) return;
  const int d = R.d;
  const double* u;
  double l, lw;
  if (q < nd) {
    u = R.du + q * d;
    l = R.dlam[q];
    lw = R.dlogw[q] - logZ;
  } else {
    const int i = (int)(q - nd);
    u = R.u + (size_t)i * d;
    l = R.lam[i];
    lw = order_value(l) + R.state->logX - log((double)R.n) - logZ;
  }
  if (theta) {
    for (int i = 0; i < d; ++i)
      theta[q * d + i] = (M.likelihood == LK_GAUSS) ? u[i] : prior_plain(M.prior, i, u[i]);
  }
  if (logl) logl[q] = l;
  if (logw) logw[q] = lw;
}

template <int NDET, int LK, bool LDS>
hipError_t launch_loglike_t(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                            const double* u, long n, double* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t lds = LDS ? (size_t)M.k_lim * (4 * sizeof(double) + NDET * sizeof(double2)) : 0;
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((k_loglike<NDET, LK, LDS>), dim3((unsigned)blocks), dim3(256), lds, st, Md, T, RB, u, n, out);
  return hipGetLastError();
}

template <int NDET, int NT, int LK, bool LDS>
hipError_t launch_slice_t(const ModelDev* Md, const Tables& T, const RBTables& RB, const RunDev& R, size_t lds,
                          hipStream_t st) {
  hipLaunchKernelGGL((k_slice<NDET, NT, LK, LDS>), dim3(R.k), dim3(NT), lds, st, Md, T, RB, R);
  return hipGetLastError();
}

template <int NDET, int NT>
hipError_t launch_slice_nt(const ModelDev* Md, const Tables& T, const RBTables& RB, const RunDev& R,
                           const LaunchCfg& C, hipStream_t st) {
  if (C.lds_tables) return launch_slice_t<NDET, NT, LK_FULL, true>(Md, T, RB, R, C.lds_bytes, st);
  return launch_slice_t<NDET, NT, LK_FULL, false>(Md, T, RB, R, C.lds_bytes, st);
}

template <int NDET>
hipError_t launch_slice_det(const ModelDev* Md, const Tables& T, const RBTables& RB, const RunDev& R,
                            const LaunchCfg& C, hipStream_t st) {
  switch (C.slice_threads) {
    case 64: return launch_slice_nt<NDET, 64>(Md, T, RB, R, C, st);
    case 128: return launch_slice_nt<NDET, 128>(Md, T, RB, R, C, st);
    default: return launch_slice_nt<NDET, 256>(Md, T, RB, R, C, st);
  }
}

size_t slice_lds_fixed() { return (size_t)(MAX_DIM * MAX_DIM + 16) * sizeof(double); }

}  // namespace

int likelihood_kind(const ModelDev& M) { return M.likelihood; }

hipError_t configure_slice(const ModelDev& M, LaunchCfg* C) {
  if (M.likelihood == LK_GAUSS) {
    C->slice_threads = 64;
    C->lds_tables = false;
    C->lds_bytes = slice_lds_fixed();
    return hipSuccess;
  }
  const long work = (long)M.k_lim * M.n_det;   // (bin, detector) terms of the widest probe
  C->slice_threads = work <= 96 ? 64 : (work <= 320 ? 128 : 256);
  const size_t tab = (size_t)M.k_lim * (4 * sizeof(double) + M.n_det * sizeof(double2));
  C->lds_tables = tab <= 64 * 1024;
  C->lds_bytes = slice_lds_fixed() + (C->lds_tables ? tab : 0);
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

hipError_t launch_init_live(const RunDev& R, hipStream_t st) {
  hipLaunchKernelGGL(k_init_live, dim3((R.n + 255) / 256), dim3(256), 0, st, R.n, R.d, R.key0, R.key1, R.u);
  return hipGetLastError();
}

hipError_t launch_loglike(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                          const double* u, long n, double* out, hipStream_t st) {
  if (M.likelihood == LK_GAUSS) return launch_loglike_t<1, LK_GAUSS, false>(M, Md, T, RB, u, n, out, st);
  const size_t tab = (size_t)M.k_lim * (4 * sizeof(double) + M.n_det * sizeof(double2));
  const bool lds = tab <= 64 * 1024;
  switch (M.n_det) {
    case 1: return lds ? launch_loglike_t<1, LK_FULL, true>(M, Md, T, RB, u, n, out, st)
                       : launch_loglike_t<1, LK_FULL, false>(M, Md, T, RB, u, n, out, st);
    case 2: return lds ? launch_loglike_t<2, LK_FULL, true>(M, Md, T, RB, u, n, out, st)
                       : launch_loglike_t<2, LK_FULL, false>(M, Md, T, RB, u, n, out, st);
    default: return lds ? launch_loglike_t<3, LK_FULL, true>(M, Md, T, RB, u, n, out, st)
                        : launch_loglike_t<3, LK_FULL, false>(M, Md, T, RB, u, n, out, st);
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
  hipLaunchKernelGGL(k_prep, dim3(1), dim3(1024), (size_t)R.n * sizeof(int), st, R);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
  if (M.likelihood == LK_GAUSS) {
    e = launch_slice_t<1, 64, LK_GAUSS, false>(Md, T, RB, R, C.lds_bytes, st);
  } else {
    switch (M.n_det) {
      case 1: e = launch_slice_det<1>(Md, T, RB, R, C, st); break;
      case 2: e = launch_slice_det<2>(Md, T, RB, R, C, st); break;
      default: e = launch_slice_det<3>(Md, T, RB, R, C, st); break;
    }
  }
  if (e != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[3], st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_term, dim3(1), dim3(1024), 0, st, R);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[4], st)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_waveform(const ModelDev& M, const ModelDev* Md, const double* theta_dev, int det, int apply_cut,
                           double* h_re, double* h_im, hipStream_t st) {
  hipLaunchKernelGGL(k_waveform, dim3((M.n_bins + 255) / 256), dim3(256), 0, st, Md, theta_dev, det, apply_cut,
                     h_re, h_im);
  return hipGetLastError();
}

hipError_t launch_final(const RunDev& R, int n_sim, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_final, dim3(1 + (n_sim > 0 ? n_sim : 0)), dim3(1024), 0, st, R, n_sim, out);
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
