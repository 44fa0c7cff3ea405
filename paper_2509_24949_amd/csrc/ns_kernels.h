// Device code of libns for gfx950 (wave64), shared by the kernel sources:
// ns_kernels.hip (host-side launchers and every non-chain kernel) and the
// ns_slice_*.hip files, each of which instantiates one group of chain
// kernels (so the groups compile in parallel).
//
//  * k_rank       bit-exact selection: the rank of every live point in the
//                 total order (order key, slot); the k lowest die.
//  * k_prep       one workgroup: evidence and prior-volume update of the k
//                 deaths, dead-point record, covariance of the live points
//                 and its Cholesky factor, survivor list, chain start points.
//  * k_slice      one workgroup per chain: the whole constrained slice walk
//                 of the iteration with the chain state uniform across the
//                 workgroup and the likelihood tables in LDS.  Each step sets
//                 up a batch of candidate probes whose positions are known in
//                 advance (the step-out points and the shrink candidates), the
//                 two halves of the workgroup computing the intrinsic and the
//                 extrinsic half of every candidate's source; the walk then
//                 evaluates independent probes in pairs, each probe's bins
//                 spread over half the workgroup and reduced once.  A
//                 separate 64-thread instantiation also counts the walk's
//                 moves for the per-iteration metrics.
//  * k_term       one workgroup: live evidence, termination flag, counters,
//                 the iteration's metrics record.
//  * k_probe_setup2 (k_probe_setup), k_probe_bins
//                 batched fused full-grid likelihood in two passes: the probe
//                 set-up (two threads per probe), then one wavefront per probe
//                 over the frequency bins with the coefficients in scalar
//                 registers.
//  * k_rb_lane    batched relative-binning likelihood in one pass: two lanes
//                 per probe walk its edges with the wavefront, the edge
//                 records (k_rb_edge_records) staged in LDS.
//  * k_loglike    batched likelihood in one pass (initial population of the
//                 full-grid and Gaussian forms).
//  * k_*_packed   the serving forms: one launch covers the chains (and the
//                 selection, preparation and termination) of every resident run.
#pragma once
#include <float.h>
#include <math.h>
#include <stdlib.h>

#include <type_traits>

#include "ns_internal.h"

namespace ns {

namespace {

constexpr double NEG_INF = -__builtin_inf();

// Value of lane i ^ 1, i ^ 2 (quad permutations), of the mirrored lane in
// the half row (8 lanes) and in the row (16 lanes), through DPP.
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
constexpr int DPP_XOR1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;

// Value of lane `src` (uniform) as a scalar.
__device__ inline double row_value(double v, int src) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), src),
                          __builtin_amdgcn_readlane(__double2loint(v), src));
}

// Wavefront sum with every lane active: a butterfly inside each row of 16
// lanes (both partners of a pair add the same two values, so every lane of
// a row holds the same row sum), then (r0 + r1) + (r2 + r3) over the rows.
// The order is fixed, so the result is reproducible and uniform.
__device__ inline double wave_sum(double v) {
  v += dpp_d<DPP_XOR1>(v);
  v += dpp_d<DPP_XOR2>(v);
  v += dpp_d<DPP_HALF_MIRROR>(v);
  v += dpp_d<DPP_MIRROR>(v);
  const double r0 = row_value(v, 0), r1 = row_value(v, 16), r2 = row_value(v, 32), r3 = row_value(v, 48);
  return (r0 + r1) + (r2 + r3);
}

__device__ inline double wave_max(double v) {
  v = fmax(v, dpp_d<DPP_XOR1>(v));
  v = fmax(v, dpp_d<DPP_XOR2>(v));
  v = fmax(v, dpp_d<DPP_HALF_MIRROR>(v));
  v = fmax(v, dpp_d<DPP_MIRROR>(v));
  const double r0 = row_value(v, 0), r1 = row_value(v, 16), r2 = row_value(v, 32), r3 = row_value(v, 48);
  return fmax(fmax(r0, r1), fmax(r2, r3));
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

// Inclusive prefix sum over the NT threads in thread order (wave shuffles,
// then the wave totals); *total receives the sum of all.  Two barriers;
// sbuf holds NT/64 values.
template <int NT, typename T>
__device__ inline T block_scan(T v, T* sbuf, T* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  __syncthreads();
  if (lane == 63) sbuf[wv] = v;
  __syncthreads();
  T off = T(0), all = T(0);
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wv) off += sbuf[w];
    all += sbuf[w];
  }
  *total = all;
  return v + off;
}

// K block-wide sums at once (two barriers); every thread receives them.
// sbuf holds K * NT/64 values.
template <int NT, int K>
__device__ inline void block_sum_k(double (&v)[K], double* sbuf) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < K; ++q) v[q] = wave_sum(v[q]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < K; ++q) sbuf[q * NW + wv] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < K; ++q) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += sbuf[q * NW + w];
    v[q] = t;
  }
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
  const double* f;      // bin k of f, f13, lnf3, fm53 at [k * ts]
  const double* f13;
  const double* lnf3;
  const double* fm53;
  int ts;
  const double2* dw;    // detector d, bin k at [k * dk + d * dd]
  const float2* dw32;   // (the same strides in float2 units)
  int dk, dd;
  const double* hpre;   // prefix sums of 4 df f^(-7/3) / S per detector
  int hstride;          // row stride of hpre
  double inv_scale;     // 1 / dw_scale of the float table
};

// LDS bytes of the staged full-grid tables.
__host__ __device__ inline size_t staged_table_bytes(int k_lim, int n_det, bool mixed) {
  return (size_t)k_lim * (4 * sizeof(double) + n_det * (sizeof(double) + (mixed ? sizeof(float2) : sizeof(double2))));
}

template <int NDET, bool MX>
__device__ inline TabView stage_tables(const ModelDev& M, const Tables& T, bool use_lds, double* lds, int tid,
                                       int nt) {
  TabView V;
  if (!use_lds) {
    V.f = T.f; V.f13 = T.f13; V.lnf3 = T.lnf3; V.fm53 = T.fm53; V.dw = T.dw; V.dw32 = T.dw32; V.hpre = T.hpre;
    V.ts = 1;
    V.dk = 1;
    V.dd = M.n_bins;
    V.hstride = M.n_bins;
    V.inv_scale = MX ? 1.0 / M.dw_scale : 1.0;
    return V;
  }
  // one record per bin: f, f^(1/3), ln f / 3, f^(-5/3), then the detectors'
  // data (double2 each, or float2 in the mixed form), so a bin is read from
  // one base address; the prefix table follows the records
  const int K = M.k_lim;
  constexpr int RD = MX ? 4 + NDET : 4 + 2 * NDET;   // doubles per record (even without MX: 16-byte aligned)
  for (int k = tid; k < K; k += nt) {
    double* rec = lds + (size_t)k * RD;
    rec[0] = T.f[k];
    rec[1] = T.f13[k];
    rec[2] = T.lnf3[k];
    rec[3] = T.fm53[k];
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
      if (MX) reinterpret_cast<float2*>(rec + 4)[d] = T.dw32[(size_t)d * M.n_bins + k];
      else reinterpret_cast<double2*>(rec + 4)[d] = T.dw[(size_t)d * M.n_bins + k];
    }
  }
  double* hp = lds + (size_t)K * RD;
  for (int i = tid; i < NDET * K; i += nt) {
    const int d = i / K, k = i - d * K;
    hp[i] = T.hpre[(size_t)d * M.n_bins + k];
  }
  V.f = lds; V.f13 = lds + 1; V.lnf3 = lds + 2; V.fm53 = lds + 3; V.ts = RD;
  V.dw = reinterpret_cast<const double2*>(lds + 4);
  V.dw32 = reinterpret_cast<const float2*>(lds + 4);
  V.dk = MX ? RD : RD / 2;      // record stride in float2 or double2 units
  V.dd = 1;
  V.hpre = hp;
  V.hstride = K;
  V.inv_scale = MX ? 1.0 / M.dw_scale : 1.0;
  return V;
}

// sin and cos of 2 pi r for |r| <= 1/2 cycles, single precision, on the
// transcendental unit (whose sine and cosine take their argument in cycles).
__device__ inline float2 sincos_cycles_f32(float r) {
  return make_float2(__builtin_amdgcn_sinf(r), __builtin_amdgcn_cosf(r));
}

// Compensated (Kahan) accumulation in single precision.
struct KahanF {
  float s = 0.0f, c = 0.0f;
  __device__ inline void add(float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
  }
};

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

// One bin's table entries: frequency terms and the detectors' whitened data.
template <int NDET, bool MX>
struct BinRow {
  double f, f13, lnf3, fm53;
  typename std::conditional<MX, float2, double2>::type D[NDET];
};

template <int NDET, bool MX>
__device__ inline BinRow<NDET, MX> load_bin(const TabView& V, int k) {
  BinRow<NDET, MX> r;
  const size_t kt = (size_t)k * V.ts;
  r.f = V.f[kt];
  r.f13 = V.f13[kt];
  r.lnf3 = V.lnf3[kt];
  r.fm53 = V.fm53[kt];
#pragma unroll
  for (int d = 0; d < NDET; ++d) {
    if constexpr (MX) r.D[d] = V.dw32[(size_t)k * V.dk + d * V.dd];
    else r.D[d] = V.dw[(size_t)k * V.dk + d * V.dd];
  }
  return r;
}

// This thread's share of <d|h> summed over detectors, for the active bins
// k = lane, lane + nl, ...:  sum_d Re[A K_d sum_k conj(Dw_dk) e^{-i Phi_dk}].
// Per detector the bin sums a_d = sum (Dr c - Di s) and b_d = sum (Dr s + Di c)
// are folded with A K_d = (kre, kim) as kre a_d + kim b_d before returning, so a
// probe needs a single reduction.  With PF the next bin's table entries are
// loaded before the current bin is computed, so that their latency overlaps
// the arithmetic (for kernels with few waves per SIMD).
template <int NDET, bool MX, bool PF = false>
__device__ inline double fullgrid_partial(const Probe& p, const TabView& V, int lane, int nl) {
  using Row = BinRow<NDET, MX>;
  [[maybe_unused]] Row nxt{};
  if constexpr (PF) {
    if (lane < p.k_act) nxt = load_bin<NDET, MX>(V, lane);
  }
  if constexpr (MX) {
    // mixed form: the phase in double, reduced to [-1/2, 1/2] cycles, then
    // float sincos and compensated float sums of the scaled data
    KahanF a[NDET], b[NDET];
    for (int k = lane; k < p.k_act; k += nl) {
      Row r;
      if constexpr (PF) {
        r = nxt;
        const int kn = k + nl < p.k_act ? k + nl : k;   // the last pass re-reads its own bin
        nxt = load_bin<NDET, MX>(V, kn);
      } else {
        r = load_bin<NDET, MX>(V, k);
      }
      const double psi = phase_cycles(p, r.f, r.f13, r.lnf3, r.fm53);
#pragma unroll
      for (int d = 0; d < NDET; ++d) {
        const double ph = fma(r.f, p.dt[d], psi);
        const float2 sc = sincos_cycles_f32((float)(ph - rint(ph)));
        const float2 D = r.D[d];
        a[d].add(fmaf(D.x, sc.y, -D.y * sc.x));
        b[d].add(fmaf(D.x, sc.x, D.y * sc.y));
      }
    }
    double part = 0.0;
#pragma unroll
    for (int d = 0; d < NDET; ++d)
      part = fma(p.kre[d], (double)a[d].s, fma(p.kim[d], (double)b[d].s, part));
    return part * V.inv_scale;
  } else {
    double a[NDET], b[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) { a[d] = 0.0; b[d] = 0.0; }
    for (int k = lane; k < p.k_act; k += nl) {
      Row r;
      if constexpr (PF) {
        r = nxt;
        const int kn = k + nl < p.k_act ? k + nl : k;
        nxt = load_bin<NDET, MX>(V, kn);
      } else {
        r = load_bin<NDET, MX>(V, k);
      }
      const double psi = phase_cycles(p, r.f, r.f13, r.lnf3, r.fm53);
#pragma unroll
      for (int d = 0; d < NDET; ++d) {
        const double2 sc_ = sincos_cycles(fma(r.f, p.dt[d], psi));
        const double sn = sc_.x, cs = sc_.y;
        const double2 D = r.D[d];
        a[d] = fma(D.x, cs, fma(-D.y, sn, a[d]));
        b[d] = fma(D.x, sn, fma(D.y, cs, b[d]));
      }
    }
    double part = 0.0;
#pragma unroll
    for (int d = 0; d < NDET; ++d) part = fma(p.kre[d], a[d], fma(p.kim[d], b[d], part));
    return part;
  }
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

// ------------------------------------------------------- relative binning
// Grid frequency f_lo + k df as a product followed by a sum (no fused
// multiply-add), the rounding the edge snapping is defined with.
__device__ inline double grid_freq(double f_lo, double df, int k) {
#pragma clang fp contract(off)
  return f_lo + (double)k * df;
}

// Edges e_b = f_lo (f_hi / f_lo)^(b / nb), snapped to the nearest grid
// frequency, the first and last pinned to the ends of the grid.
__global__ void k_rb_edges(const ModelDev* __restrict__ Mp, int nb, int* edge, double* fe, double* fe13,
                           double* lnfe3, double* fem53) {
  const ModelDev& M = *Mp;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > nb) return;
  const double f_hi = grid_freq(M.f_lo, M.df, M.n_bins - 1);
  const double raw = M.f_lo * pow(f_hi / M.f_lo, (double)e / nb);
  int k = (int)floor((raw - M.f_lo) / M.df + 0.5);
  k = k < 0 ? 0 : (k > M.n_bins - 1 ? M.n_bins - 1 : k);
  if (e == 0) k = 0;
  if (e == nb) k = M.n_bins - 1;
  const double f = grid_freq(M.f_lo, M.df, k);
  const double lf = log(f);
  edge[e] = k;
  fe[e] = f;
  fe13[e] = cbrt(f);
  lnfe3[e] = lf / 3.0;
  fem53[e] = exp(-5.0 / 3.0 * lf);
}

// Fiducial phases at the edges, bin centres and widths, 1 / (A0 K0_det).
__global__ void k_rb_fiducial(const ModelDev* __restrict__ Mp, const double* theta, int nb, const double* fe,
                              const double* fe13, const double* lnfe3, const double* fem53, double* phi0,
                              double2* g0, double* fm, double* inv_w) {
  const ModelDev& M = *Mp;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > nb) return;
  Phys s;
  phys_from_theta(M, theta, &s);
  Probe P;
  probe_from_phys(M, s, nullptr, &P);
  const double psi = phase_cycles(P, fe[e], fe13[e], lnfe3[e], fem53[e]);
  for (int d = 0; d < M.n_det; ++d) phi0[d * (nb + 1) + e] = fma(fe[e], P.dt[d], psi);
  if (e < nb) {
    fm[e] = 0.5 * (fe[e] + fe[e + 1]);
    inv_w[e] = 1.0 / (fe[e + 1] - fe[e]);
  }
  if (e == 0) {
    for (int d = 0; d < M.n_det; ++d) {
      const double den = P.kre[d] * P.kre[d] + P.kim[d] * P.kim[d];
      g0[d] = make_double2(P.kre[d] / den, -P.kim[d] / den);
    }
  }
}

// Summary sums, one thread per (detector, coarse bin), accumulated over the
// bin's fine bins in frequency order; the running sums are kept per fine bin.
__global__ void k_rb_sums(const ModelDev* __restrict__ Mp, Tables T, const double* hw, const double* theta, int nb,
                          const int* edge, const double* fm, double2* A0, double2* A1, double* B0, double* B1,
                          double2* cA0, double2* cA1, double* cB0, double* cB1) {
  const ModelDev& M = *Mp;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int d = blockIdx.y;
  if (b >= nb) return;
  Phys s;
  phys_from_theta(M, theta, &s);
  Probe P;
  probe_from_phys(M, s, nullptr, &P);
  const double kr = P.kre[d], ki = P.kim[d];
  const double k2 = kr * kr + ki * ki;
  const int first = edge[b], last = (b < nb - 1) ? edge[b + 1] - 1 : edge[nb];
  const double fmb = fm[b];
  double s0r = 0, s0i = 0, s1r = 0, s1i = 0, t0 = 0, t1 = 0;
  for (int k = first; k <= last; ++k) {
    const size_t o = (size_t)d * M.n_bins + k;
    const double f = T.f[k];
    const double ph = fma(f, P.dt[d], phase_cycles(P, f, T.f13[k], T.lnf3[k], T.fm53[k]));
    const double2 sc_ = sincos_cycles(ph);
    const double sn = sc_.x, cs = sc_.y;
    // A0 K0 e^{-i Phi0}: the fiducial strain without f^(-7/6) (carried by dw)
    const double er = kr * cs + ki * sn, ei = ki * cs - kr * sn;
    const double2 D = T.dw[o];
    const double ar = D.x * er + D.y * ei, ai = D.x * ei - D.y * er;   // conj(dw) * K0 e^{-i Phi0}
    const double bk = k2 * hw[o];
    const double x = f - fmb;
    s0r += ar; s0i += ai;
    s1r += ar * x; s1i += ai * x;
    t0 += bk; t1 += bk * x;
    cA0[o] = make_double2(s0r, s0i);
    cA1[o] = make_double2(s1r, s1i);
    cB0[o] = t0;
    cB1[o] = t1;
  }
  const size_t q = (size_t)d * nb + b;
  A0[q] = make_double2(s0r, s0i);
  A1[q] = make_double2(s1r, s1i);
  B0[q] = t0;
  B1[q] = t1;
}

// This thread's share of lambda for one probe under relative binning.  Phase
// 1: the ratio r_d(e) = h(e) / h0(e) = A K_d / (A0 K0_d) e^{-i (Phi_d - Phi0_d)}
// at the edges e = tid, tid + nt, ... into LDS.  Phase 2: per coarse bin
// b = tid, ...: r0 = (r_b + r_{b+1}) / 2, r1 = (r_{b+1} - r_b) / (e_{b+1} - e_b),
// Re(A0 r0 + A1 r1) - 1/2 [B0 |r0|^2 + 2 B1 Re(conj(r0) r1)]; bins whose first
// fine bin is above f_ISCO are skipped and the straddling bin uses the sums
// up to its last active fine bin.  Contains one workgroup barrier.
// Relative-binning tables staged in LDS by a chain workgroup (doubles from a
// 16-byte aligned base): edge frequencies and their powers, fiducial phases,
// 1 / bin width, edge indices, then the bin sums (double, or float in the
// mixed form).  The cumulative sums of the straddling bin stay in HBM.
__host__ __device__ inline size_t rb_stage_doubles(int nb, int n_det, bool mixed) {
  const size_t ne = nb + 1, nbd = (size_t)n_det * nb;
  size_t o = (4 + (size_t)n_det) * ne + nb + (ne + 1) / 2;
  o += o & 1;
  return o + (mixed ? 2 * nbd + 2 * ((nbd + 1) / 2) : 6 * nbd);
}

template <int NDET, bool MX>
__device__ inline RBTables stage_rb(const RBTables& B, double* lds, int tid, int nt) {
  RBTables V = B;
  const int nb = B.nb, ne = nb + 1, nbd = NDET * nb;
  double* fe = lds;
  double* fe13 = fe + ne;
  double* lnfe3 = fe13 + ne;
  double* fem53 = lnfe3 + ne;
  double* phi0 = fem53 + ne;
  double* inv_w = phi0 + NDET * ne;
  int* edge = reinterpret_cast<int*>(inv_w + nb);
  size_t o = (size_t)(4 + NDET) * ne + nb + (ne + 1) / 2;
  o += o & 1;
  for (int e = tid; e < ne; e += nt) {
    fe[e] = B.fe[e];
    fe13[e] = B.fe13[e];
    lnfe3[e] = B.lnfe3[e];
    fem53[e] = B.fem53[e];
    edge[e] = B.edge[e];
#pragma unroll
    for (int d = 0; d < NDET; ++d) phi0[d * ne + e] = B.phi0[d * ne + e];
  }
  for (int b = tid; b < nb; b += nt) inv_w[b] = B.inv_w[b];
  V.fe = fe; V.fe13 = fe13; V.lnfe3 = lnfe3; V.fem53 = fem53; V.phi0 = phi0; V.inv_w = inv_w; V.edge = edge;
  if constexpr (MX) {
    float2* a0 = reinterpret_cast<float2*>(lds + o);
    float2* a1 = a0 + nbd;
    float* b0 = reinterpret_cast<float*>(a1 + nbd);
    float* b1 = b0 + 2 * ((nbd + 1) / 2);
    for (int i = tid; i < nbd; i += nt) {
      a0[i] = B.A0f[i]; a1[i] = B.A1f[i]; b0[i] = B.B0f[i]; b1[i] = B.B1f[i];
    }
    V.A0f = a0; V.A1f = a1; V.B0f = b0; V.B1f = b1;
  } else {
    double2* a0 = reinterpret_cast<double2*>(lds + o);
    double2* a1 = a0 + nbd;
    double* b0 = reinterpret_cast<double*>(a1 + nbd);
    double* b1 = b0 + nbd;
    for (int i = tid; i < nbd; i += nt) {
      a0[i] = B.A0[i]; a1[i] = B.A1[i]; b0[i] = B.B0[i]; b1[i] = B.B1[i];
    }
    V.A0 = a0; V.A1 = a1; V.B0 = b0; V.B1 = b1;
  }
  return V;
}

// Coarse bins a probe with k_act active grid bins reads: the bins b < nb
// whose first fine bin edge[b] lies below k_act.  Edges increase, so a
// ballot over the wavefront counts them 64 at a time and stops at the first
// incomplete group (every lane takes part; the result is uniform).
__device__ inline int rb_active_bins(const RBTables& B, int k_act, int lane) {
  int n_act = 0;
  for (int b0 = 0; b0 < B.nb; b0 += 64) {
    const int b = b0 + lane;
    const int c = __popcll(__ballot(b < B.nb && B.edge[b] < k_act));
    n_act += c;
    if (c < 64) break;
  }
  return n_act;
}

// Relative-binning likelihood of one probe, evaluated by one wavefront
// (every lane calls it; the result is uniform).  With n_act active coarse
// bins the probe reads edges 0 .. n_act.  They are taken in chunks of 63
// bins: lane l computes the ratio r_d(e) = h(e) / h0(e)
// = A K_d / (A0 K0_d) e^{-2 pi i (Phi_d(e) - Phi0_d(e))} at edge e = c0 + l for
// every detector, receives r_d(e + 1) from lane l + 1, and (l < 63) adds
// coarse bin b = e:  r0 = (r_b + r_{b+1}) / 2, r1 = (r_{b+1} - r_b) / (f_{b+1} - f_b),
// Re(A0 r0 + A1 r1) - 1/2 [B0 |r0|^2 + 2 B1 Re(conj(r0) r1)].  The bin that
// straddles f_ISCO (its last fine bin at or above k_act) uses the sums
// accumulated up to fine bin k_act - 1, loaded before the edge arithmetic.
// *n_edges receives the edges read (n_act + 1, or 0 when no bin is active).
template <int NDET, bool MX>
__device__ inline double rb_wave(const Probe& p, const RBTables& B, int n_bins, int lane, int* n_edges) {
  using RT = typename std::conditional<MX, float, double>::type;
  const int nb = B.nb, ne = nb + 1;
  const int n_act = rb_active_bins(B, p.k_act, lane);
  *n_edges = n_act > 0 ? n_act + 1 : 0;
  if (n_act == 0) return 0.0;
  const int sb = n_act - 1;
  const int sb_last = (sb < nb - 1) ? B.edge[sb + 1] - 1 : B.edge[nb];
  const bool straddle = sb_last >= p.k_act;
  double part = 0.0;
  for (int c0 = 0; c0 < n_act; c0 += 63) {
    const int e = c0 + lane;
    const bool has_edge = e <= n_act;
    const bool has_bin = lane < 63 && e < n_act;
    const bool cum = straddle && has_bin && e == sb;
    // the phase at this lane's edge, shared by the detectors
    double f = 0.0, psi = 0.0;
    if (has_edge) {
      f = B.fe[e];
      psi = phase_cycles(p, f, B.fe13[e], B.lnfe3[e], B.fem53[e]);
    }
    const RT iw = has_bin ? (RT)B.inv_w[e] : (RT)0;
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
      // ratio at this lane's edge ...
      RT rr = (RT)0, ri = (RT)0;
      if (has_edge) {
        const double2 g = B.g0[d];
        const double gr = p.kre[d] * g.x - p.kim[d] * g.y, gi = p.kre[d] * g.y + p.kim[d] * g.x;
        const double dph = fma(f, p.dt[d], psi) - B.phi0[d * ne + e];
        if constexpr (MX) {
          const float2 sc = sincos_cycles_f32((float)(dph - rint(dph)));
          const float fr = (float)gr, fi = (float)gi;
          rr = fmaf(fr, sc.y, fi * sc.x);
          ri = fmaf(fi, sc.y, -fr * sc.x);
        } else {
          const double2 sc = sincos_cycles(dph);
          rr = gr * sc.y + gi * sc.x;
          ri = gi * sc.y - gr * sc.x;
        }
      }
      // ... and at the next edge, from the next lane
      const RT nr = __shfl_down(rr, 1), ni = __shfl_down(ri, 1);
      if (has_bin) {
        RT a0r, a0i, a1r, a1i, b0, b1;
        if (cum) {
          // the straddling bin: the sums up to its last active fine bin
          const size_t q = (size_t)d * n_bins + p.k_act - 1;
          const double2 a0 = B.cA0[q], a1 = B.cA1[q];
          a0r = (RT)a0.x; a0i = (RT)a0.y; a1r = (RT)a1.x; a1i = (RT)a1.y;
          b0 = (RT)B.cB0[q]; b1 = (RT)B.cB1[q];
        } else if constexpr (MX) {
          const size_t q = (size_t)d * nb + e;
          const float2 a0 = B.A0f[q], a1 = B.A1f[q];
          a0r = a0.x; a0i = a0.y; a1r = a1.x; a1i = a1.y;
          b0 = B.B0f[q]; b1 = B.B1f[q];
        } else {
          const size_t q = (size_t)d * nb + e;
          const double2 a0 = B.A0[q], a1 = B.A1[q];
          a0r = a0.x; a0i = a0.y; a1r = a1.x; a1i = a1.y;
          b0 = B.B0[q]; b1 = B.B1[q];
        }
        const RT half = (RT)0.5, two = (RT)2;
        const RT r0r = half * (rr + nr), r0i = half * (ri + ni);
        const RT r1r = (nr - rr) * iw, r1i = (ni - ri) * iw;
        const RT dh = (a0r * r0r - a0i * r0i) + (a1r * r1r - a1i * r1i);
        const RT hh = b0 * (r0r * r0r + r0i * r0i) + two * b1 * (r0r * r1r + r0i * r1i);
        part += (double)(dh - half * hh);
      }
    }
  }
  return wave_sum(part);
}

// Batched relative-binning likelihood, one probe per lane.  Every lane sets
// up its probe and finds its active coarse bins (the bins whose first fine
// bin lies below its k_act, by bisection of the ascending edge indices); the
// wavefront then walks the edges e = 0, 1, ... together, reading one record
// per edge (built at run construction, k_rb_edge_records) from a copy the
// block stages in LDS (every lane at the same address, the next edge's
// record loading while this edge is computed), and a lane whose probe has
// fewer active bins idles from its last edge on.
//
// The linear model of coarse bin b, Re(A0 r0 + A1 r1) - 1/2 [B0 |r0|^2 +
// 2 B1 Re(conj(r0) r1)] with r0 = (r_b + r_{b+1})/2 and r1 = (r_{b+1} - r_b) w_b
// (w_b the inverse bin width), equals
//   Re(P_b r_b + Q_b r_{b+1}) - 1/2 [C_b |r_b|^2 + D_b |r_{b+1}|^2 + E_b Re(conj(r_b) r_{b+1})]
// with P = A0/2 - A1 w, Q = A0/2 + A1 w, C = B0/4 - B1 w, D = B0/4 + B1 w,
// E = B0/2 (the cross term of 2 B1 Re(conj(r0) r1) cancels).  Summed over
// consecutive bins, edge e contributes Re(W_e r_e) - 1/2 [G_e |r_e|^2 +
// E_{e-1} Re(conj(r_{e-1}) r_e)] with W_e = Q_{e-1} + P_e and G_e = D_{e-1} + C_e,
// so the record of edge e holds W, G and E_{e-1} per detector, and a lane's
// first edge takes only the right-hand parts P, C (kept in a second table)
// and its last edge has them taken off again.  The bin that straddles
// f_ISCO is left out of the walk and added afterwards in the bin form from
// the sums accumulated up to fine bin k_act - 1, with the ratios at its two
// edges recomputed.  No cross-lane reduction is needed.
template <int NDET, bool MX>
__device__ inline void rb_ratio(const Probe& p, const double* gr, const double* gi, double psi, double f,
                                double phi0, int d,
                                typename std::conditional<MX, float, double>::type* rr,
                                typename std::conditional<MX, float, double>::type* ri) {
  const double dph = fma(f, p.dt[d], psi) - phi0;
  if constexpr (MX) {
    const float2 sc = sincos_cycles_f32((float)(dph - rint(dph)));
    const float fr = (float)gr[d], fi = (float)gi[d];
    *rr = fmaf(fr, sc.y, fi * sc.x);
    *ri = fmaf(fi, sc.y, -fr * sc.x);
  } else {
    const double2 sc = sincos_cycles(dph);
    *rr = gr[d] * sc.y + gi[d] * sc.x;
    *ri = gi[d] * sc.y - gr[d] * sc.x;
  }
}

template <typename RT>
__device__ inline RT rb_bin_term(RT rr, RT ri, RT nr, RT ni, RT iw, RT a0r, RT a0i, RT a1r, RT a1i, RT b0, RT b1) {
  const RT half = (RT)0.5, two = (RT)2;
  const RT r0r = half * (rr + nr), r0i = half * (ri + ni);
  const RT r1r = (nr - rr) * iw, r1i = (ni - ri) * iw;
  const RT dh = (a0r * r0r - a0i * r0i) + (a1r * r1r - a1i * r1i);
  const RT hh = b0 * (r0r * r0r + r0i * r0i) + two * b1 * (r0r * r1r + r0i * r1i);
  return dh - half * hh;
}

// Edge e's coefficients for detector d: W (complex), G, E_{e-1} and the
// right-hand parts P_e (complex), C_e (bins outside 0 .. nb - 1 contribute 0).
struct RBEdgeCoef {
  double wr, wi, g, ep, pr, pi, c;
};

__device__ inline RBEdgeCoef rb_edge_coef(const RBTables& B, int e, int d) {
  const int nb = B.nb;
  RBEdgeCoef k{0, 0, 0, 0, 0, 0, 0};
  if (e >= 1) {                           // bin e - 1 on the left: Q, D, E
    const int b = e - 1;
    const size_t q = (size_t)d * nb + b;
    const double w = B.inv_w[b];
    const double2 a0 = B.A0[q], a1 = B.A1[q];
    k.wr = fma(a1.x, w, 0.5 * a0.x);
    k.wi = fma(a1.y, w, 0.5 * a0.y);
    k.g = fma(B.B1[q], w, 0.25 * B.B0[q]);
    k.ep = 0.5 * B.B0[q];
  }
  if (e < nb) {                           // bin e on the right: P, C
    const size_t q = (size_t)d * nb + e;
    const double w = B.inv_w[e];
    const double2 a0 = B.A0[q], a1 = B.A1[q];
    k.pr = fma(-a1.x, w, 0.5 * a0.x);
    k.pi = fma(-a1.y, w, 0.5 * a0.y);
    k.c = fma(-B.B1[q], w, 0.25 * B.B0[q]);
    k.wr += k.pr;
    k.wi += k.pi;
    k.g += k.c;
  }
  return k;
}

// Edge records of k_rb_lane: per edge its frequency terms and fiducial
// phases and, per detector, W (2), G, E_{e-1}; then per edge and detector the
// right-hand parts P (2), C.  The mixed form keeps the coefficients as floats.
__host__ __device__ constexpr int rb_lane_rec_doubles(int n_det, bool mixed) {
  return mixed ? ((4 + 3 * n_det + 1) & ~1) : ((4 + 5 * n_det + 1) & ~1);
}
__host__ __device__ constexpr int rb_lane_right_doubles(int n_det, bool mixed) {
  return mixed ? ((3 * n_det + 1) / 2) : 3 * n_det;
}

template <int NDET, bool MX>
struct RBEdge {
  using RT = typename std::conditional<MX, float, double>::type;
  double f, f13, lnf3, fm53;
  double phi0[NDET];
  RT wr[NDET], wi[NDET], g[NDET], ep[NDET];
};

// Builds the edge records (one thread per edge): records [nb+1][RD], then
// the right-hand parts [nb+1][RR].
template <int NDET, bool MX>
__global__ void k_rb_edge_records(RBTables B, double* erec) {
  using RT = typename std::conditional<MX, float, double>::type;
  constexpr int RD = rb_lane_rec_doubles(NDET, MX), RR = rb_lane_right_doubles(NDET, MX);
  const int nb = B.nb, ne = nb + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double* r = erec + (size_t)e * RD;
  double* right = erec + (size_t)ne * RD + (size_t)e * RR;
  for (int k = 0; k < RD; ++k) r[k] = 0.0;
  for (int k = 0; k < RR; ++k) right[k] = 0.0;
  r[0] = B.fe[e]; r[1] = B.fe13[e]; r[2] = B.lnfe3[e]; r[3] = B.fem53[e];
  RT* c = reinterpret_cast<RT*>(r + 4 + NDET);
  RT* rt = reinterpret_cast<RT*>(right);
#pragma unroll
  for (int d = 0; d < NDET; ++d) {
    r[4 + d] = B.phi0[d * ne + e];
    const RBEdgeCoef k = rb_edge_coef(B, e, d);
    c[4 * d] = (RT)k.wr; c[4 * d + 1] = (RT)k.wi; c[4 * d + 2] = (RT)k.g; c[4 * d + 3] = (RT)k.ep;
    rt[3 * d] = (RT)k.pr; rt[3 * d + 1] = (RT)k.pi; rt[3 * d + 2] = (RT)k.c;
  }
}

// The record of edge e (from the block's LDS copy or from the device array).
template <int NDET, bool MX>
__device__ inline void rb_lane_load(const double* recs, int e, RBEdge<NDET, MX>& x) {
  using RT = typename std::conditional<MX, float, double>::type;
  constexpr int RD = rb_lane_rec_doubles(NDET, MX);
  const double* r = recs + (size_t)e * RD;
  x.f = r[0]; x.f13 = r[1]; x.lnf3 = r[2]; x.fm53 = r[3];
  const RT* c = reinterpret_cast<const RT*>(r + 4 + NDET);
#pragma unroll
  for (int d = 0; d < NDET; ++d) {
    x.phi0[d] = r[4 + d];
    x.wr[d] = c[4 * d]; x.wi[d] = c[4 * d + 1]; x.g[d] = c[4 * d + 2]; x.ep[d] = c[4 * d + 3];
  }
}

// The right-hand parts P, C of edge e for detector d.
template <int NDET, bool MX>
__device__ inline void rb_lane_right(const double* recs, int ne, int e, int d,
                                     typename std::conditional<MX, float, double>::type* pr,
                                     typename std::conditional<MX, float, double>::type* pi,
                                     typename std::conditional<MX, float, double>::type* c) {
  using RT = typename std::conditional<MX, float, double>::type;
  const RT* rt = reinterpret_cast<const RT*>(recs + (size_t)ne * rb_lane_rec_doubles(NDET, MX) +
                                             (size_t)e * rb_lane_right_doubles(NDET, MX));
  *pr = rt[3 * d]; *pi = rt[3 * d + 1]; *c = rt[3 * d + 2];
}

// One edge of the walk: the ratios r_e and the edge's terms; first: a lane's
// first edge, which takes only the right-hand parts (pr0, pi0, c0).
template <int NDET, bool MX>
__device__ inline void rb_lane_edge(const Probe& p, const double* gr, const double* gi, const RBEdge<NDET, MX>& x,
                                    bool first, const typename std::conditional<MX, float, double>::type* pr0,
                                    const typename std::conditional<MX, float, double>::type* pi0,
                                    const typename std::conditional<MX, float, double>::type* c0,
                                    typename std::conditional<MX, float, double>::type* pvr,
                                    typename std::conditional<MX, float, double>::type* pvi, double& part) {
  using RT = typename std::conditional<MX, float, double>::type;
  const double psi = phase_cycles(p, x.f, x.f13, x.lnf3, x.fm53);
  RT acc = (RT)0;
#pragma unroll
  for (int dd = 0; dd < NDET; ++dd) {
    RT rr, ri;
    rb_ratio<NDET, MX>(p, gr, gi, psi, x.f, x.phi0[dd], dd, &rr, &ri);
    const RT wr = first ? pr0[dd] : x.wr[dd], wi = first ? pi0[dd] : x.wi[dd], g = first ? c0[dd] : x.g[dd];
    const RT m2 = rr * rr + ri * ri;
    const RT cross = pvr[dd] * rr + pvi[dd] * ri;          // Re(conj(r_{e-1}) r_e); 0 at a first edge
    acc += (wr * rr - wi * ri) - (RT)0.5 * (g * m2 + x.ep[dd] * cross);
    pvr[dd] = rr;
    pvi[dd] = ri;
  }
  part += (double)acc;
}

template <int NDET, bool MX, bool LDS, int H>
__global__ __launch_bounds__(256) void k_rb_lane(const ModelDev* __restrict__ Mp, RBTables RB,
                                                 const double* __restrict__ u, long n, double* __restrict__ out,
                                                 int* __restrict__ terms) {
  using RT = typename std::conditional<MX, float, double>::type;
  constexpr int PW = 64 / H;                       // probes per wavefront
  constexpr int RD = rb_lane_rec_doubles(NDET, MX);
  extern __shared__ double smem[];
  const ModelDev& M = *Mp;
  const int lane = threadIdx.x & 63;
  const int half = lane / PW;                      // 0: lower lane of the probe, 1: upper
  const long i = ((long)blockIdx.x * 4 + (threadIdx.x >> 6)) * PW + (lane % PW);
  const bool own = i < n;
  const int nb = RB.nb, ne = nb + 1;
  // the edge records and indices first: their loads overlap the probe set-up
  const size_t rec_words = (size_t)ne * (RD + rb_lane_right_doubles(NDET, MX));
  const double* recs = RB.erec;
  const int* edge = RB.edge;
  if (LDS) {
    for (size_t w = threadIdx.x; w < rec_words; w += 256) smem[w] = RB.erec[w];
    int* se = reinterpret_cast<int*>(smem + rec_words);
    for (int w = threadIdx.x; w < ne; w += 256) se[w] = RB.edge[w];
    recs = smem;
    edge = se;
  }
  const int d = M.n_dim;
  const long src = own ? i : 0;
  double y[MAX_DIM];
#pragma unroll
  for (int q = 0; q < MAX_DIM; ++q) y[q] = (q < d) ? u[src * d + q] : 0.0;
  const size_t staged = LDS ? rec_words + (size_t)(ne + 1) / 2 : 0;
  Probe pr;
  if constexpr (H == 2) {
    // the probe's two lanes set up its intrinsic and extrinsic halves side by side
    ProbeRec* rec = reinterpret_cast<ProbeRec*>(smem + staged) + ((threadIdx.x >> 6) * PW + lane % PW);
    if (half == 0) probe_intrinsic(M, y, rec);
    else probe_extrinsic<NDET>(M, y, rec);
    __syncthreads();
    pr = probe_from_rec<NDET>(*rec, false);
  } else {
    make_probe(M, nullptr, y, &pr);
    if (LDS) __syncthreads();
  }
  int n_act = 0;
  if (own) {
    int lo = 0, hi = nb;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (edge[mid] < pr.k_act) lo = mid + 1;
      else hi = mid;
    }
    n_act = lo;
  }
  const int sb = n_act - 1;
  bool straddle = false;
  if (n_act > 0) {
    const int sb_last = (sb < nb - 1) ? edge[sb + 1] - 1 : edge[nb];
    straddle = sb_last >= pr.k_act;
  }
  // the walk takes bins 0 .. last_edge - 1 from edges 0 .. last_edge
  const int last_edge = straddle ? sb : sb + 1;
  // this lane's edges: first .. last
  int first = 0, last = last_edge;
  if constexpr (H == 2) {
    int mx = last_edge;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    const int mid = (mx + 1) >> 1;
    if (half == 0) last = min(last_edge, mid);
    else first = mid;
  }
  double gr[NDET], gi[NDET];
#pragma unroll
  for (int dd = 0; dd < NDET; ++dd) {
    const double2 g = RB.g0[dd];
    gr[dd] = pr.kre[dd] * g.x - pr.kim[dd] * g.y;
    gi[dd] = pr.kre[dd] * g.y + pr.kim[dd] * g.x;
  }
  double part = 0.0;
  RT pvr[NDET], pvi[NDET], p0r[NDET], p0i[NDET], c0[NDET];
  const int e0 = min(first, nb);
#pragma unroll
  for (int dd = 0; dd < NDET; ++dd) {
    pvr[dd] = (RT)0;
    pvi[dd] = (RT)0;
    rb_lane_right<NDET, MX>(recs, ne, e0, dd, &p0r[dd], &p0i[dd], &c0[dd]);
  }
  auto load = [&](int t, RBEdge<NDET, MX>& x) { rb_lane_load<NDET, MX>(recs, min(first + t, nb), x); };
  // step t takes edge first + t; two records in flight, the next edge's
  // loads issued before this edge's arithmetic
  const int steps = last - first;                  // this lane's last step (negative: none)
  RBEdge<NDET, MX> xa, xb;
  load(0, xa);
  load(1, xb);
  if (0 <= steps) rb_lane_edge<NDET, MX>(pr, gr, gi, xa, true, p0r, p0i, c0, pvr, pvi, part);
  for (int t = 1; __builtin_amdgcn_ballot_w64(t <= steps) != 0; t += 2) {
    load(t + 1, xa);
    if (t <= steps) rb_lane_edge<NDET, MX>(pr, gr, gi, xb, false, p0r, p0i, c0, pvr, pvi, part);
    if (__builtin_amdgcn_ballot_w64(t + 1 <= steps) == 0) break;
    load(t + 2, xb);
    if (t + 1 <= steps) rb_lane_edge<NDET, MX>(pr, gr, gi, xa, false, p0r, p0i, c0, pvr, pvi, part);
  }
  if (0 <= steps) {
    // the last edge's right-hand parts belong to a bin this lane does not take
    RT acc = (RT)0;
#pragma unroll
    for (int dd = 0; dd < NDET; ++dd) {
      RT qr, qi, qc;
      rb_lane_right<NDET, MX>(recs, ne, last, dd, &qr, &qi, &qc);
      acc += (qr * pvr[dd] - qi * pvi[dd]) - (RT)0.5 * qc * (pvr[dd] * pvr[dd] + pvi[dd] * pvi[dd]);
    }
    part -= (double)acc;
  }
  if (straddle && half == 0) {
    // the straddling bin sb: ratios at its edges sb and sb + 1, sums up to fine bin k_act - 1
    const RT iw = (RT)RB.inv_w[sb];
    const double f0 = RB.fe[sb], f1 = RB.fe[sb + 1];
    const double psi0 = phase_cycles(pr, f0, RB.fe13[sb], RB.lnfe3[sb], RB.fem53[sb]);
    const double psi1 = phase_cycles(pr, f1, RB.fe13[sb + 1], RB.lnfe3[sb + 1], RB.fem53[sb + 1]);
#pragma unroll
    for (int dd = 0; dd < NDET; ++dd) {
      RT r0, i0, r1, i1;
      rb_ratio<NDET, MX>(pr, gr, gi, psi0, f0, RB.phi0[dd * ne + sb], dd, &r0, &i0);
      rb_ratio<NDET, MX>(pr, gr, gi, psi1, f1, RB.phi0[dd * ne + sb + 1], dd, &r1, &i1);
      const size_t q = (size_t)dd * M.n_bins + pr.k_act - 1;
      const double2 a0 = RB.cA0[q], a1 = RB.cA1[q];
      part += (double)rb_bin_term<RT>(r0, i0, r1, i1, iw, (RT)a0.x, (RT)a0.y, (RT)a1.x, (RT)a1.y, (RT)RB.cB0[q],
                                      (RT)RB.cB1[q]);
    }
  }
  if constexpr (H == 2) part += __shfl_down(part, 32, 64);
  if (own && half == 0) {
    out[i] = part;
    if (terms) terms[i] = n_act > 0 ? n_act + 1 : 0;
  }
}

// Float copies for the mixed form.
__global__ __launch_bounds__(1024) void k_noise_loglike(const double* __restrict__ dre, const double* __restrict__ dim,
                                                       const double* __restrict__ psd, long n, double df,
                                                       double* out) {
  __shared__ double sbuf[1024];
  double acc = 0.0;
  for (long i = threadIdx.x; i < n; i += 1024) {
    const double v = psd[i] / (4.0 * df);
    acc += -log(2.0 * PI * v) - (dre[i] * dre[i] + dim[i] * dim[i]) / (2.0 * v);
  }
  acc = block_sum<1024>(acc, sbuf);
  if (threadIdx.x == 0) *out = acc;
}

__global__ void k_to_float2(const double2* src, float2* dst, size_t n, double scale) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = make_float2((float)(src[i].x * scale), (float)(src[i].y * scale));
}

__global__ void k_to_float1(const double* src, float* dst, size_t n, double scale) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)(src[i] * scale);
}

// ---------------------------------------------------------- batched lambda
// Each wavefront takes 64 consecutive probes: lane l sets up probe base + l,
// then the wave evaluates the probes one at a time over the bins.
template <int NDET, int LK, bool LDS>
__global__ __launch_bounds__(256) void k_loglike(const ModelDev* __restrict__ Mp, Tables T, RBTables RB,
                                                 const double* __restrict__ u, long n, double* __restrict__ out,
                                                 int* __restrict__ terms) {
  extern __shared__ double smem[];
  const ModelDev& M = *Mp;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  TabView V{};
  if (lk_full(LK)) {
    V = stage_tables<NDET, lk_mixed(LK)>(M, T, LDS, smem, tid, 256);
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
    int nterm = 0;
    if (LK == LK_GAUSS) {
      mine = gauss_lambda(M, y);
    } else {
      Probe pr;
      make_probe(M, T.hpre, y, &pr);
      mine = 0.0;
      const int cnt = (n - base) < 64 ? (int)(n - base) : 64;
      for (int p = 0; p < cnt; ++p) {
        const Probe pb = probe_from_lane<NDET>(pr, p);
        const double tot = wave_sum(fullgrid_partial<NDET, lk_mixed(LK)>(pb, V, lane, 64));
        if (lane == p) mine = tot - 0.5 * pb.hh;
      }
      nterm = pr.k_act;
    }
    if (i < n) out[i] = mine;
    if (terms && i < n) terms[i] = nterm;
  }
}

// Two-pass form of the batched full-grid likelihood: the per-probe source
// set-up runs one thread per probe and stores the coefficients; the bin
// pass then runs one wavefront per probe with the coefficients in scalar
// registers, so the bin loop keeps few vector registers and many waves
// per SIMD hide its latency.
__global__ __launch_bounds__(256) void k_probe_setup(const ModelDev* __restrict__ Mp, const double* __restrict__ hpre,
                                                     const double* __restrict__ u, long n, Probe* __restrict__ P,
                                                     int* __restrict__ terms) {
  const ModelDev& M = *Mp;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int d = M.n_dim;
  double y[MAX_DIM];
#pragma unroll
  for (int q = 0; q < MAX_DIM; ++q) y[q] = (q < d) ? u[i * d + q] : 0.0;
  Probe pr;
  make_probe(M, hpre, y, &pr);
  P[i] = pr;
  if (terms) terms[i] = pr.k_act;
}

// Set-up pass of the full-grid batch for the 11-parameter models: two
// threads per probe, one computing the intrinsic half of its source and
// the other the extrinsic half (as the chain kernel's candidates do).  The
// block's unit-cube points are read into LDS with coalesced loads, and the
// finished coefficient records leave through LDS, so consecutive threads
// store consecutive 8-byte words.
constexpr int SETUP2_PROBES = 128;    // probes per 256-thread block

__host__ __device__ inline size_t setup2_lds_bytes() {
  return SETUP2_PROBES * (MAX_DIM * sizeof(double) + sizeof(ProbeRec) + sizeof(Probe));
}

template <int NDET>
__global__ __launch_bounds__(256) void k_probe_setup2(const ModelDev* __restrict__ Mp, const double* __restrict__ hpre,
                                                      const double* __restrict__ u, long n, Probe* __restrict__ P,
                                                      int* __restrict__ terms) {
  extern __shared__ double smem[];
  const ModelDev& M = *Mp;
  const int tid = threadIdx.x;
  const int d = M.n_dim;
  const long p0 = (long)blockIdx.x * SETUP2_PROBES;
  const int np = (int)min((long)SETUP2_PROBES, n - p0);
  double* su = smem;                                                    // [np][d]
  ProbeRec* recs = reinterpret_cast<ProbeRec*>(smem + SETUP2_PROBES * MAX_DIM);
  Probe* out = reinterpret_cast<Probe*>(recs + SETUP2_PROBES);
  for (int e = tid; e < np * d; e += 256) su[e] = u[p0 * d + e];
  __syncthreads();
  const int j = tid & (SETUP2_PROBES - 1);
  if (j < np) {
    double y[MAX_DIM];
#pragma unroll
    for (int q = 0; q < MAX_DIM; ++q) y[q] = (q < d) ? su[j * d + q] : 0.0;
    ProbeRec* rec = recs + j;
    if (tid < SETUP2_PROBES) {
      const int ka = probe_intrinsic(M, y, rec);
#pragma unroll
      for (int dd = 0; dd < NDET; ++dd) rec->hk[dd] = ka > 0 ? hpre[(size_t)dd * M.n_bins + ka - 1] : 0.0;
    } else {
      probe_extrinsic<NDET>(M, y, rec);
    }
  }
  __syncthreads();
  if (tid < np) {
    out[tid] = probe_from_rec<NDET>(recs[tid], true);
    if (terms) terms[p0 + tid] = recs[tid].k_act;
  }
  __syncthreads();
  static_assert(sizeof(Probe) % 8 == 0, "records move as 8-byte words");
  const int words = np * (int)(sizeof(Probe) / 8);
  const double* src = reinterpret_cast<const double*>(out);
  double* dst = reinterpret_cast<double*>(P + p0);
  for (int w = tid; w < words; w += 256) dst[w] = src[w];
}

template <int NDET, int LK, bool LDS>
// 1024 threads share one staged copy of the tables, so a CU holds eight
// waves per SIMD.
__global__ __launch_bounds__(1024) void k_probe_bins(const ModelDev* __restrict__ Mp, Tables T,
                                                     const Probe* __restrict__ P, long n, double* __restrict__ out) {
  extern __shared__ double smem[];
  const ModelDev& M = *Mp;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const TabView V = stage_tables<NDET, lk_mixed(LK)>(M, T, LDS, smem, tid, 1024);
  if (LDS) __syncthreads();
  for (long p = (long)blockIdx.x * 16 + wv; p < n; p += (long)gridDim.x * 16) {
    const Probe pb = P[p];
    const double tot = wave_sum(fullgrid_partial<NDET, lk_mixed(LK)>(pb, V, lane, 64));
    if (lane == 0) out[p] = tot - 0.5 * pb.hh;
  }
}


// ---------------------------------------------------------------- select
// Rank of element i in the total order (order key, index), one wavefront.
__device__ inline void rank_element(const double* __restrict__ lam, int n, int k, int* rank, int* dead, double* lstar,
                                    int i, int lane) {
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

__global__ __launch_bounds__(256) void k_rank(const double* __restrict__ lam, int n, int k, int* rank, int* dead,
                                              double* lstar, const int* done) {
  if (done && *done) return;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= n) return;
  rank_element(lam, n, k, rank, dead, lstar, i, lane);
}

// ------------------------------------------------------------- iteration prep
// One workgroup of 1024 threads; s_surv: n ints of LDS (survivor list).
constexpr int PCH = 1024;             // live points per chunk of the mean and covariance passes

// One workgroup of 1024 threads.  spts holds a chunk of live points by
// coordinate (all of them when n <= PCH) and afterwards the survivor list.
__device__ void prep_body(const RunDev& R) {
  __shared__ double sbuf[1024];
  __shared__ double spts[MAX_DIM * PCH];
  int* s_surv = reinterpret_cast<int*>(spts);
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
  // the iteration's evaluations-per-step histogram, which the slice chains
  // add to
  if (tid < PROBE_HIST && it < R.trace_cap) R.trace[it].hist[tid] = 0;

  // ---- evidence: the j-th death shrinks log X by 1/(n-j); its weight is the
  // shell between consecutive volumes, X_{j-1} (1 - e^{-1/(n-j)}).
  const int C = (k + 1023) / 1024;
  const int jb = tid * C, je = min(k, jb + C);
  double csum = 0.0;
  for (int j = jb; j < je; ++j) csum += 1.0 / (double)(n - j);
  double total;                                        // sum of 1/(n-j) over the batch
  const double incl = block_scan<1024, double>(csum, sbuf, &total);
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
    R.dlam[q] = lraw;
    R.dlogx[q] = lxn;
    R.dlogw[q] = lw;
    R.diter[q] = it;
    R.dslot[q] = slot;
    R.dnlive[q] = n - j;
    mloc = fmax(mloc, lw);
    lx = lxn;
  }
  // the dead points' coordinates, copied with independent loads
  for (int idx = tid; idx < k * d; idx += 1024) {
    const int j = idx / d, i = idx - j * d;
    R.du[(nd0 + j) * d + i] = R.u[(size_t)R.dead[j] * d + i];
  }
  double m = block_max<1024>(mloc, sbuf);
  m = fmax(m, logZ0);
  double s12[2] = {0.0, 0.0};
  if (m > NEG_INF) {
    for (int j = jb; j < je; ++j) {
      const double lw = R.dlogw[nd0 + j];
      if (lw > NEG_INF) {
        const double e = exp(lw - m);
        s12[0] += e;
        s12[1] += e * order_value(R.dlam[nd0 + j]);
      }
    }
  }
  block_sum_k<1024, 2>(s12, sbuf);
  const double s1 = s12[0], s2 = s12[1];
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
  // The points pass through LDS in chunks of PCH, one row per coordinate,
  // read with coalesced loads: first for the mean (a group of 1024/d threads
  // per coordinate), then, centred, for the covariance.
  {
    const int G1 = 1024 / d;
    const int mi = tid / G1, msub = tid - mi * G1;
    double ms = 0.0;
    for (int j0 = 0; j0 < n; j0 += PCH) {
      const int cnt = min(PCH, n - j0);
      __syncthreads();                // the previous chunk has been read
      for (int idx = tid; idx < cnt * d; idx += 1024) {
        const int jj = idx / d, i = idx - jj * d;
        spts[i * PCH + jj] = R.u[(size_t)j0 * d + idx];
      }
      __syncthreads();
      if (mi < d)
        for (int jj = msub; jj < cnt; jj += G1) ms += spts[mi * PCH + jj];
    }
    sbuf[tid] = ms;
    __syncthreads();
    if (tid < d) {
      double t = 0.0;
      for (int q = 0; q < G1; ++q) t += sbuf[tid * G1 + q];
      smean[tid] = t / n;
    }
    __syncthreads();
  }
  // lower-triangle entry e -> (a, b), a >= b, row-major: a group of G
  // threads sums each entry over a strided share of every chunk (the chunk
  // of the mean pass is still in LDS when n <= PCH), and the group's partial
  // sums meet in LDS at the end
  const int E = d * (d + 1) / 2;
  const int G = 1024 / E;
  const int lane = tid & 63, wv = tid >> 6;
  const int eg = tid / G, sub = tid - eg * G;
  int ea = 0, eb = 0;
  if (eg < E) {
    int r = eg;
    while (r > ea) { r -= ea + 1; ++ea; }
    eb = r;
  }
  const double ma = smean[ea], mb = smean[eb];
  double cs = 0.0;
  for (int j0 = 0; j0 < n; j0 += PCH) {
    const int cnt = min(PCH, n - j0);
    if (n > PCH) {
      __syncthreads();                // the previous chunk has been read
      for (int idx = tid; idx < cnt * d; idx += 1024) {
        const int jj = idx / d, i = idx - jj * d;
        spts[i * PCH + jj] = R.u[(size_t)j0 * d + idx];
      }
      __syncthreads();
    }
    if (eg < E) {
      const double* ra = spts + ea * PCH;
      const double* rb = spts + eb * PCH;
      for (int jj = sub; jj < cnt; jj += G) cs += (ra[jj] - ma) * (rb[jj] - mb);
    }
  }
  sbuf[tid] = cs;
  __syncthreads();
  if (tid < E) {
    int a = 0, r = tid;
    while (r > a) { r -= a + 1; ++a; }
    const int b = r;
    double c = 0.0;
    for (int q = 0; q < G; ++q) c += sbuf[tid * G + q];
    c /= (double)(n - 1);
    scov[a * d + b] = c;
    scov[b * d + a] = c;
  }
  __syncthreads();
  if (wv == 0) {
    // Cholesky factor, one row per lane (row j broadcast from lane j); on
    // failure add 1e-12 tr/d to the diagonal and retry
    double L[MAX_DIM];
    bool ok = false;
    for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
      if (attempt == 1) {
        double tr = 0.0;
        for (int i = 0; i < d; ++i) tr += scov[i * d + i];
        if (lane < d) scov[lane * d + lane] += 1e-12 * tr / d;
      }
      ok = true;
#pragma unroll
      for (int q = 0; q < MAX_DIM; ++q) L[q] = 0.0;
#pragma unroll
      for (int j = 0; j < MAX_DIM; ++j) {
        if (j < d) {
          double s = lane < d ? scov[lane * d + j] : 0.0;
#pragma unroll
          for (int q = 0; q < j; ++q) s -= L[q] * lane_d(L[q], j);
          const double diag = lane_d(s, j);
          ok = ok && diag > 0.0;
          const double ljj = sqrt(fmax(diag, 0.0));
          L[j] = (lane == j) ? ljj : (lane > j && ljj > 0.0 ? s / ljj : 0.0);
        }
      }
    }
    if (lane < d) {
#pragma unroll
      for (int q = 0; q < MAX_DIM; ++q)
        if (q < d) R.chol[lane * d + q] = ok ? (q <= lane ? L[q] : 0.0) : (q == lane ? 1e-6 : 0.0);
    }
  }

  // ---- survivors in ascending slot order, then the chain start points
  const int C2 = (n + 1023) / 1024;
  const int ib = tid * C2, ie = min(n, ib + C2);
  int cnt = 0;
  for (int i = ib; i < ie; ++i) cnt += (R.rank[i] >= k);
  int all_surv;
  const int icl = block_scan<1024, int>(cnt, sint, &all_surv);
  int pos = icl - cnt;
  for (int i = ib; i < ie; ++i)
    if (R.rank[i] >= k) {
      s_surv[pos] = i;
      R.surv[pos] = i;   // the random-walk chains draw their proposal pairs from it
      ++pos;
    }
  __syncthreads();
  const int ns = n - k;
  for (int j = tid; j < k; j += 1024) {
    u64x4 b = philox((uint64_t)it, (uint64_t)j, 0, purpose_word(P_PICK, 0), R.key0, R.key1);
    const int idx = (int)floor(unif53(b.x[0]) * (double)ns);
    R.start[j] = s_surv[idx < ns ? idx : ns - 1];
  }
}

__global__ __launch_bounds__(1024) void k_prep(RunDev R) { prep_body(R); }


// ------------------------------------------------------------ slice chains
// Candidate batches of the chain kernel: NC candidates per batch, each set
// up by two threads (the intrinsic and the extrinsic half of the probe).
// Slots [0, SO) hold left step-out points, [SO, 2 SO) right ones, the rest
// the first SC shrink candidates of each bracket the step-out can end in
// with at most H-1 steps per side.  A step outside the batch (more step-outs
// or shrink attempts) costs a further batch, so the slots go where steps
// need them: a side rarely steps out more than twice at these widths, and a
// step's rejected shrink candidates run past six far more often (measured:
// 0.6 expansions and 1.7 rejected shrink candidates per step).
template <int NC> struct SliceBatch {
  static constexpr int SO = NC >= 128 ? NC / 8 : 4;
  static constexpr int H = NC >= 64 ? 3 : 2;
  static constexpr int SC = NC >= 128 ? 10 : 6;
  static_assert(2 * SO + H * H * SC <= NC, "batch layout");
};

// Dynamic LDS of the chain kernel (doubles), in order: Cholesky factor,
// reduction slots, directions and uniforms of a chunk of steps, the batch
// (probe records, positions, Gaussian values or fallback uniforms, in-cube
// flags), the chain position, then the likelihood tables (full grid, when
// they fit) or the edge ratios (relative binning).
constexpr int SL_CHUNK = 16;                          // steps drawn per chunk
constexpr int SL_PSTRIDE = (int)((sizeof(ProbeRec) + 15) / 16) * 2;   // doubles per stored record
constexpr int SL_NU = 14;                             // uniforms per step: width, split, 12 shrink
constexpr int SL_CNT = PROBE_HIST + 4 + 4 * SL_CHUNK;  // ints of the walk's move counters
__host__ __device__ constexpr size_t slice_fixed_doubles(int nt, bool mv) {
  return MAX_DIM * MAX_DIM + 16 + SL_CHUNK * MAX_DIM + SL_CHUNK * SL_NU + (size_t)(nt / 2) * SL_PSTRIDE + nt + nt +
         nt / 4 + 16 + (mv ? SL_CNT / 2 : 0);
}

// One workgroup of NT threads runs chain j = blockIdx.x for all n_steps
// steps.  The random numbers and tuned directions of a chunk of steps are
// drawn up front, lane-parallel.  Each step then sets up one batch of NT/2
// candidates in parallel (each fixed in advance: the step-out points and,
// under the hypothesis that earlier candidates are rejected, the shrink
// sequence of every likely bracket); the first half of the workgroup
// computes the intrinsic half of every candidate's probe while the second
// half computes the extrinsic one.  All threads then walk the batch in the
// sequential order of the algorithm and split every probe's frequency bins.
// Rarer outcomes fall back to further batches.  MV: also count the walk's
// moves (bracket expansions, rejected shrink candidates, moved steps and
// the evaluations of each step) for the iteration's metrics record; the
// counting is a separate instantiation so that the other kernels carry none
// of it.
template <int NDET, int NT, int LK, bool LDS, bool MV = false>
__device__ void slice_body(const ModelDev& M, const Tables& T, const RBTables& RB, const RunDev& R, int j,
                           double* smem) {
  constexpr int NW = NT / 64;
  constexpr int NC = NT / 2;         // candidates per batch
  constexpr int FB = NC < 32 ? NC : 32;   // candidates per fallback batch
  using BL = SliceBatch<NC>;
  DevState* S = R.state;
  if (S->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int d = R.d;
  const uint64_t t = (uint64_t)S->iter;
  const double lstar = S->lstar;
  double* sL = smem;
  double* sred = sL + MAX_DIM * MAX_DIM;
  double* sDir = sred + 16;
  double* sU = sDir + SL_CHUNK * MAX_DIM;
  double* sP = sU + SL_CHUNK * SL_NU;
  double* sT = sP + NC * SL_PSTRIDE;
  double* sG = sT + NT;
  unsigned long long* sMask = reinterpret_cast<unsigned long long*>(sG + NT);   // in-cube bits per 64 candidates
  double* sX = sG + NT + NT / 4;     // chain position
  // the walk's moves: steps by the evaluations they made ([0, PROBE_HIST),
  // the last bin for that many or more), bracket expansions, rejected shrink
  // candidates, steps that moved, and the evaluations made before the
  // current chunk; then one record per step of the chunk (evaluations so
  // far, expansions, rejected shrink candidates, moved), written by thread 0
  // as the step ends and folded into the counts once per chunk
  int* sCnt = reinterpret_cast<int*>(sX + 16);
  int* sStep = sCnt + PROBE_HIST + 4;
  double* stab = sX + 16 + (MV ? SL_CNT / 2 : 0);
  for (int i = tid; i < d * d; i += NT) sL[i] = R.chol[i];
  if constexpr (MV)
    for (int i = tid; i < SL_CNT; i += NT) sCnt[i] = 0;
  TabView V{};
  if (lk_full(LK)) V = stage_tables<NDET, lk_mixed(LK)>(M, T, LDS, stab, tid, NT);
  // relative binning: the tables, staged in LDS when LDS is set
  RBTables RBv = RB;
  if constexpr (lk_rb(LK) && LDS) RBv = stage_rb<NDET, lk_mixed(LK)>(RB, stab, tid, NT);

  int buf = 0;
  int nprobe = 0;
  long long nbins = 0;
  const int start = R.start[j];
  for (int i = tid; i < d; i += NT) sX[i] = R.u[(size_t)start * d + i];
  double lx = R.lam[start];
  const int nbd = (d + 3) >> 2;      // DIR blocks per step
  const double w = R.width;

  // candidate c = tid mod NC of a batch, at position tt along dir (valid:
  // the slot is used; unused slots are marked outside the cube); threads
  // below NC compute the intrinsic half of its probe, the others the
  // extrinsic half
  const int cand = tid % NC;
  const bool intrinsic_half = tid < NC;
  auto setup = [&](bool valid, double tt, const double* dir) {
    // all MAX_DIM slots of the position and direction rows are read (slots
    // from d on are masked), so the loads issue together instead of one
    // dependent round trip per coordinate
    double xr[MAX_DIM], dr[MAX_DIM];
#pragma unroll
    for (int i = 0; i < MAX_DIM; ++i) {
      xr[i] = sX[i];
      dr[i] = dir[i];
    }
    double y[MAX_DIM];
    bool cin = valid;
#pragma unroll
    for (int i = 0; i < MAX_DIM; ++i) {
      // a periodic coordinate is taken modulo 1 and is always inside
      const bool per = (M.periodic >> i) & 1u;
      const double yi = cube_coord(M.periodic, i, fma(tt, dr[i], xr[i]));
      const bool act = i < d;
      y[i] = act ? yi : 0.0;
      cin = cin && (!act || per || (yi >= 0.0 && yi <= 1.0));
    }
    if (!cin) {
#pragma unroll
      for (int i = 0; i < MAX_DIM; ++i) y[i] = 0.5;   // a harmless point; never evaluated
    }
    const unsigned long long m = __ballot(cin);
    ProbeRec* rec = reinterpret_cast<ProbeRec*>(sP + cand * SL_PSTRIDE);
    if (intrinsic_half) {
      if (LK == LK_GAUSS) {
        sG[cand] = gauss_lambda(M, y);
      } else {
        const int ka = probe_intrinsic(M, y, rec);
        if constexpr (lk_full(LK)) {
          // the prefix-table entries <h|h> needs, read here once rather than
          // by every evaluating thread
#pragma unroll
          for (int dd = 0; dd < NDET; ++dd) rec->hk[dd] = ka > 0 ? V.hpre[(size_t)dd * V.hstride + ka - 1] : 0.0;
        }
      }
      sT[cand] = tt;
      if (lane == 0) sMask[cand >> 6] = m;
    } else if (LK != LK_GAUSS) {
      probe_extrinsic<NDET>(M, y, rec);
    }
  };
  // After a batch's barrier every wave keeps the in-cube bits and the
  // positions of the batch in registers; the walk then reads a candidate's
  // with scalar operations instead of LDS round trips.
  unsigned long long mk0 = 0, mk1 = 0;
  double tr0 = 0.0, tr1 = 0.0;
  auto load_batch = [&]() {
    mk0 = sMask[0];
    tr0 = sT[lane];
    if constexpr (NC > 64) {
      mk1 = sMask[1];
      tr1 = sT[64 + lane];
    }
  };
  auto inside = [&](int q) -> bool { return ((q < 64 ? mk0 : mk1) >> (q & 63)) & 1ull; };
  auto ttq = [&](int q) -> double { return lane_d(q < 64 ? tr0 : tr1, q & 63); };
  // lambda of batch candidate q (all threads; contains workgroup barriers)
  auto eval = [&](int q) -> double {
    ++nprobe;
    if (LK == LK_GAUSS) return sG[q];
    const Probe pb = probe_from_rec<NDET>(*reinterpret_cast<const ProbeRec*>(sP + q * SL_PSTRIDE), lk_full(LK));
    if constexpr (lk_rb(LK)) {
      // every wave evaluates the probe (no exchange needed); terms: the edges read
      int ne;
      const double tot = rb_wave<NDET, lk_mixed(LK)>(pb, RBv, M.n_bins, lane, &ne);
      nbins += ne;
      return tot;
    }
    double* rb = sred + buf * (NW + 4);
    double tot = wave_sum(fullgrid_partial<NDET, lk_mixed(LK), true>(pb, V, tid, NT));
    if constexpr (NW > 1) {
      if (lane == 0) rb[wv] = tot;
      __syncthreads();
      tot = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) tot += rb[w2];
      buf ^= 1;
    }
    // terms: the active bins
    nbins += pb.k_act;
    return tot - 0.5 * pb.hh;
  };
  // Full grid with two or more waves: lambdas of two candidates at once
  // (q < 0: none), the first half of the workgroup summing the bins of q1,
  // the second those of q2, one barrier for both.  Relative binning with two
  // or more waves: NW candidates at once, one per wavefront.  Nothing is
  // counted here: the walk counts the evaluations the sequential algorithm
  // makes.
  constexpr bool PAIR = lk_full(LK) && NW >= 2;
  constexpr bool MULTI = lk_rb(LK) && NW >= 2;
  auto rec = [&](int q) -> const ProbeRec& { return *reinterpret_cast<const ProbeRec*>(sP + q * SL_PSTRIDE); };
  auto count = [&](int terms) {   // the probe's active bins or relative-binning edges
    ++nprobe;
    nbins += terms;
  };
  auto eval2 = [&](int q1, int q2, double* l1, double* l2, int* k1, int* k2) {
    if constexpr (PAIR) {
      constexpr int HW = NW / 2;
      const bool second = tid >= NT / 2;
      const int q = second ? q2 : q1;
      double* rb = sred + buf * (NW + 4);
      double part = 0.0, hh = 0.0, kact = 0.0;
      if (q >= 0) {
        const Probe pb = probe_from_rec<NDET>(rec(q), true);
        part = fullgrid_partial<NDET, lk_mixed(LK), true>(pb, V, second ? tid - NT / 2 : tid, NT / 2);
        hh = pb.hh;
        kact = (double)pb.k_act;
      }
      const double tot = wave_sum(part);
      if (lane == 0) rb[wv] = tot;
      if (lane == 0 && wv % HW == 0) {
        rb[NW + (second ? 1 : 0)] = hh;
        rb[NW + 2 + (second ? 1 : 0)] = kact;
      }
      __syncthreads();
      double t1 = 0.0, t2 = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < HW; ++w2) {
        t1 += rb[w2];
        t2 += rb[HW + w2];
      }
      *l1 = t1 - 0.5 * rb[NW];
      *l2 = t2 - 0.5 * rb[NW + 1];
      *k1 = (int)rb[NW + 2];
      *k2 = (int)rb[NW + 3];
      buf ^= 1;
    }
  };
  // Relative binning: wave w evaluates candidate qof(w) (q < 0: none); one
  // barrier shares the NW lambdas and term counts, which the caller reads
  // from the returned LDS slots (res[w], res[NW + w]) until the next call
  // but one (the slots alternate between two buffers).
  auto evalw = [&](auto qof) -> const double* {
    double* rb = sred + buf * (2 * NW);
    if constexpr (MULTI) {
      const int q = qof(wv);
      if (q >= 0) {
        const Probe pb = probe_from_rec<NDET>(rec(q), false);
        int ne;
        const double l = rb_wave<NDET, lk_mixed(LK)>(pb, RBv, M.n_bins, lane, &ne);
        if (lane == 0) {
          rb[wv] = l;
          rb[NW + wv] = (double)ne;
        }
      }
      __syncthreads();
      buf ^= 1;
    }
    return rb;
  };

  // wave 0 folds the step records of a finished chunk of ns steps into the
  // counts (after a barrier that follows the chunk's last step)
  auto fold = [&](int ns) {
    if (wv == 0 && lane < ns) {
      const int* r = sStep + 4 * lane;
      const int before = lane == 0 ? sCnt[PROBE_HIST + 3] : sStep[4 * (lane - 1)];
      const int pe = r[0] - before;
      atomicAdd(&sCnt[pe < PROBE_HIST - 1 ? pe : PROBE_HIST - 1], 1);
      atomicAdd(&sCnt[PROBE_HIST], r[1]);
      atomicAdd(&sCnt[PROBE_HIST + 1], r[2]);
      atomicAdd(&sCnt[PROBE_HIST + 2], r[3]);
      if (lane == ns - 1) sCnt[PROBE_HIST + 3] = r[0];
    }
  };

  for (int s0 = 0; s0 < R.m; s0 += SL_CHUNK) {
    const int cs = (R.m - s0) < SL_CHUNK ? (R.m - s0) : SL_CHUNK;
    // ---- draw the chunk: per step nbd direction blocks (two Box-Muller
    // pairs each), the width block and three shrink blocks
    __syncthreads();
    if constexpr (MV)
      if (s0 > 0) fold(SL_CHUNK);
    const int per = nbd + 1 + (SL_NU - 2) / 4;
    for (int bI = tid; bI < cs * per; bI += NT) {
      const int sl = bI / per, r = bI - sl * per;
      const uint64_t s = (uint64_t)(s0 + sl);
      uint64_t pw;
      if (r < nbd) pw = purpose_word(P_DIR, (uint64_t)r);
      else if (r == nbd) pw = purpose_word(P_WIDTH, 0);
      else pw = purpose_word(P_SHRINK, (uint64_t)(r - nbd - 1));
      const u64x4 b = philox(t, (uint64_t)j, s, pw, R.key0, R.key1);
      const double u0 = unif53(b.x[0]), u1 = unif53(b.x[1]), u2 = unif53(b.x[2]), u3 = unif53(b.x[3]);
      if (r < nbd) {
        const double ra = sqrt(-2.0 * log(1.0 - u0));
        const double2 ea = sincos_cycles(u1);
        const double rb = sqrt(-2.0 * log(1.0 - u2));
        const double2 eb = sincos_cycles(u3);
        double* zr = sDir + sl * MAX_DIM + 4 * r;
        if (4 * r + 0 < d) zr[0] = ra * ea.y;
        if (4 * r + 1 < d) zr[1] = ra * ea.x;
        if (4 * r + 2 < d) zr[2] = rb * eb.y;
        if (4 * r + 3 < d) zr[3] = rb * eb.x;
      } else if (r == nbd) {
        sU[sl * SL_NU + 0] = u0;
        sU[sl * SL_NU + 1] = u1;
      } else {
        double* ur = sU + sl * SL_NU + 2 + 4 * (r - nbd - 1);
        ur[0] = u0; ur[1] = u1; ur[2] = u2; ur[3] = u3;
      }
    }
    __syncthreads();
    // directions L z / |z|, one thread per step (the thread owns the row)
    for (int sl = tid; sl < cs; sl += NT) {
      // whole rows are loaded (entries past d or past the diagonal are
      // masked; every index stays below MAX_DIM^2), so each row's loads
      // issue together
      double z[MAX_DIM];
#pragma unroll
      for (int i = 0; i < MAX_DIM; ++i) z[i] = sDir[sl * MAX_DIM + i];
#pragma unroll
      for (int i = 0; i < MAX_DIM; ++i) z[i] = (i < d) ? z[i] : 0.0;
      double nrm = 0.0;
#pragma unroll
      for (int i = 0; i < MAX_DIM; ++i)
        if (i < d) nrm += z[i] * z[i];
      nrm = sqrt(nrm);
#pragma unroll
      for (int a = 0; a < MAX_DIM; ++a) {
        if (a < d) {
          double lr[MAX_DIM];
#pragma unroll
          for (int b = 0; b < MAX_DIM; ++b) lr[b] = sL[a * d + b];
          double acc = 0.0;
#pragma unroll
          for (int b = 0; b < MAX_DIM; ++b)
            if (b <= a) acc += lr[b] * z[b];
          sDir[sl * MAX_DIM + a] = acc / nrm;
        }
      }
    }
    __syncthreads();

    for (int sl = 0; sl < cs; ++sl) {
      const int s = s0 + sl;
      const double* dir = sDir + sl * MAX_DIM;
      const double* su = sU + sl * SL_NU;
      double sur[SL_NU];             // this step's uniforms, in registers
#pragma unroll
      for (int i = 0; i < SL_NU; ++i) sur[i] = su[i];
      double lo = -w * sur[0], hi = lo + w;
      int J = (int)floor(R.max_stepout * sur[1]);
      int K = R.max_stepout - 1 - J;

      // ---- the combined batch
      __syncthreads();
      {
        // both kinds of position are formed branch-free (x + (-w) is x - w
        // exactly), and each lane keeps the one its slot needs
        const bool so = cand < 2 * BL::SO;
        const bool valid = cand < 2 * BL::SO + BL::H * BL::H * BL::SC;
        // step-out point: `steps` whole widths beyond the initial bracket
        const bool left = cand < BL::SO;
        const int steps = left ? cand : cand - BL::SO;
        const double ws = left ? -w : w;
        double ts = left ? lo : hi;
#pragma unroll
        for (int q = 0; q < BL::SO - 1; ++q) ts = q < steps ? ts + ws : ts;
        // shrink point: attempt c of bracket hypothesis h
        const int hc = so ? 0 : cand - 2 * BL::SO;
        const int h = hc / BL::SC, c = hc - BL::SC * h;
        const int na = h / BL::H, nbh = h - BL::H * na;
        double l2 = lo, h2 = hi;
#pragma unroll
        for (int q = 0; q < BL::H - 1; ++q) {
          l2 = q < na ? l2 + (-w) : l2;
          h2 = q < nbh ? h2 + w : h2;
        }
        double tsh = 0.0;
#pragma unroll
        for (int q = 0; q < BL::SC; ++q) {
          if (q <= c) {
            tsh = fma(sur[2 + q], h2 - l2, l2);
            if (tsh < 0.0) l2 = tsh; else h2 = tsh;
          }
        }
        const double tt = !valid ? 0.0 : (so ? ts : tsh);
        setup(valid, tt, dir);
      }
      __syncthreads();
      load_batch();
      bool combined = true;        // the batch in LDS is the combined one

      // ---- step out, left then right (the order of the sequential algorithm)
      int na = 0, nh = 0;          // successful steps per side
      int uL = 0, uR = 0;          // batch points of each side already walked
      if constexpr (MULTI) {
        // up to NW points per round, shared between the sides (a side's later
        // points under the hypothesis that its earlier ones are accepted);
        // a side's points after its first rejection are not counted
        for (;;) {
          if (J > 0 && uL < BL::SO && !inside(uL)) J = 0;
          if (K > 0 && uR < BL::SO && !inside(BL::SO + uR)) K = 0;
          auto can_l = [&](int i) { return J > i && uL + i < BL::SO && inside(uL + i); };
          auto can_r = [&](int i) { return K > i && uR + i < BL::SO && inside(BL::SO + uR + i); };
          int nl = 0, nr = 0;
          while (nl + nr < NW) {
            const bool okl = can_l(nl), okr = can_r(nr);
            if (!okl && !okr) break;
            if (okl && (nl <= nr || !okr)) ++nl; else ++nr;
          }
          if (nl + nr == 0) break;
          const double* res = evalw([&](int w2) {
            return w2 < nl ? uL + w2 : (w2 < nl + nr ? BL::SO + uR + (w2 - nl) : -1);
          });
          for (int i = 0; i < nl; ++i) {
            count((int)res[NW + i]);
            if (res[i] > lstar) { lo -= w; --J; ++na; ++uL; } else { J = 0; break; }
          }
          for (int i = 0; i < nr; ++i) {
            count((int)res[NW + nl + i]);
            if (res[nl + i] > lstar) { hi += w; --K; ++nh; ++uR; } else { K = 0; break; }
          }
        }
      } else if constexpr (PAIR) {
        // the two sides are independent: walk them together, one pair of
        // probes per round, while their next points are in the batch; the
        // probes evaluated are exactly those of the left-then-right walk
        for (;;) {
          int qL = (J > 0 && uL < BL::SO) ? uL : -1;
          int qR = (K > 0 && uR < BL::SO) ? BL::SO + uR : -1;
          if (qL >= 0 && !inside(qL)) { J = 0; qL = -1; }
          if (qR >= 0 && !inside(qR)) { K = 0; qR = -1; }
          if (qL < 0 && qR < 0) break;
          double lL, lR;
          int kL, kR;
          eval2(qL, qR, &lL, &lR, &kL, &kR);
          if (qL >= 0) {
            count(kL);
            if (lL > lstar) { lo -= w; --J; ++na; ++uL; } else { J = 0; }
          }
          if (qR >= 0) {
            count(kR);
            if (lR > lstar) { hi += w; --K; ++nh; ++uR; } else { K = 0; }
          }
        }
      }
      for (int side = 0; side < 2; ++side) {
        int& budget = side == 0 ? J : K;
        int& done_steps = side == 0 ? na : nh;
        int first = side == 0 ? 0 : BL::SO;   // batch slot of this side's next candidate
        int have = combined ? BL::SO : 0;     // candidates of this side in the batch in LDS
        int used = combined ? (side == 0 ? uL : uR) : 0;
        while (budget > 0) {
          if (used == have) {
            // further step-out points of this side: a batch of FB
            __syncthreads();
            double tt = side == 0 ? lo : hi;
            if (cand < FB)
              for (int q = 0; q < cand; ++q) tt = side == 0 ? tt - w : tt + w;
            setup(cand < FB, tt, dir);
            __syncthreads();
            load_batch();
            combined = false;
            first = 0;
            have = FB;
            used = 0;
          }
          const int q = first + used;
          if (!inside(q)) { budget = 0; break; }
          if (!(eval(q) > lstar)) { budget = 0; break; }
          if (side == 0) lo -= w; else hi += w;
          --budget;
          ++done_steps;
          ++used;
        }
      }

      if constexpr (MV)
        if (tid == 0) sStep[4 * sl + 1] = na + nh;

      // ---- shrink
      int a = 0;                   // shrink attempts rejected so far
      bool accepted = false;
      if (MULTI && combined && na < BL::H && nh < BL::H) {
        // attempts a .. a+NW-1 together (each under the hypothesis that the
        // earlier ones are rejected); a probe is counted only where the
        // sequential walk makes it
        const int base = 2 * BL::SO + BL::SC * (BL::H * na + nh);
        while (!accepted && a < BL::SC && a < R.max_shrink) {
          const int lim = (BL::SC < R.max_shrink ? BL::SC : R.max_shrink) - a;
          const int nq = lim < NW ? lim : NW;
          bool any = false;
          for (int w2 = 0; w2 < nq; ++w2) any = any || inside(base + a + w2);
          const double* res = nullptr;
          if (any) res = evalw([&](int w2) { return (w2 < nq && inside(base + a + w2)) ? base + a + w2 : -1; });
          for (int i = 0; i < nq; ++i) {
            const double tq = ttq(base + a);
            if (inside(base + a)) {
              count((int)res[NW + i]);
              const double li = res[i];
              if (li > lstar) {
                if (tid < d) sX[tid] = cube_coord(M.periodic, tid, fma(tq, dir[tid], sX[tid]));
                lx = li;
                accepted = true;
                break;
              }
            }
            if (tq < 0.0) lo = tq; else hi = tq;
            ++a;
          }
        }
      } else if (PAIR && combined && na < BL::H && nh < BL::H) {
        // attempts a and a+1 together (a+1 under the hypothesis that a is
        // rejected); a probe is counted only where the sequential walk makes it
        const int base = 2 * BL::SO + BL::SC * (BL::H * na + nh);
        while (a < BL::SC && a < R.max_shrink) {
          const int q1 = base + a;
          const bool two = a + 1 < BL::SC && a + 1 < R.max_shrink;
          const int q2 = two ? q1 + 1 : -1;
          const bool in1 = inside(q1), in2 = two && inside(q2);
          double l1 = NEG_INF, l2 = NEG_INF;
          int k1 = 0, k2 = 0;
          if (in1 || in2) eval2(in1 ? q1 : -1, in2 ? q2 : -1, &l1, &l2, &k1, &k2);
          const double t1 = ttq(q1);
          if (in1) {
            count(k1);
            if (l1 > lstar) {
              if (tid < d) sX[tid] = cube_coord(M.periodic, tid, fma(t1, dir[tid], sX[tid]));
              lx = l1;
              accepted = true;
              break;
            }
          }
          if (t1 < 0.0) lo = t1; else hi = t1;
          ++a;
          if (!two) continue;
          const double t2 = ttq(q2);
          if (in2) {
            count(k2);
            if (l2 > lstar) {
              if (tid < d) sX[tid] = cube_coord(M.periodic, tid, fma(t2, dir[tid], sX[tid]));
              lx = l2;
              accepted = true;
              break;
            }
          }
          if (t2 < 0.0) lo = t2; else hi = t2;
          ++a;
        }
      } else if (combined && na < BL::H && nh < BL::H) {
        const int base = 2 * BL::SO + BL::SC * (BL::H * na + nh);
        for (; a < BL::SC && a < R.max_shrink; ++a) {
          const int q = base + a;
          const double tt = ttq(q);
          if (inside(q)) {
            const double ly = eval(q);
            if (ly > lstar) {
              if (tid < d) sX[tid] = cube_coord(M.periodic, tid, fma(tt, dir[tid], sX[tid]));
              lx = ly;
              accepted = true;
              break;
            }
          }
          if (tt < 0.0) lo = tt; else hi = tt;
        }
      }
      while (!accepted && a < R.max_shrink) {
        // a batch of FB shrink candidates from the current bracket: the
        // uniforms of attempts a .. a+FB-1 are drawn lane-parallel, then the
        // bracket recursion under rejection is walked once
        __syncthreads();
        if (tid < FB) {
          const int aa = a + tid;
          double ua;
          if (aa < SL_NU - 2) {
            ua = su[2 + aa];
          } else {
            const u64x4 b = philox(t, (uint64_t)j, (uint64_t)s, purpose_word(P_SHRINK, (uint64_t)(aa >> 2)),
                                   R.key0, R.key1);
            const int ws = aa & 3;
            ua = unif53(ws == 0 ? b.x[0] : ws == 1 ? b.x[1] : ws == 2 ? b.x[2] : b.x[3]);
          }
          sG[tid] = ua;
        }
        __syncthreads();
        {
          double l2 = lo, h2 = hi, tl = 0.0;
          for (int q = 0; q < FB; ++q) {
            const double tq = fma(sG[q], h2 - l2, l2);
            if (q == cand) tl = tq;
            if (tq < 0.0) l2 = tq; else h2 = tq;
          }
          __syncthreads();   // sG is reused by the Gaussian test likelihood
          setup(cand < FB, tl, dir);
        }
        __syncthreads();
        load_batch();
        for (int q = 0; q < FB && a < R.max_shrink; ++q, ++a) {
          const double tt = ttq(q);
          if (inside(q)) {
            const double ly = eval(q);
            if (ly > lstar) {
              if (tid < d) sX[tid] = cube_coord(M.periodic, tid, fma(tt, dir[tid], sX[tid]));
              lx = ly;
              accepted = true;
              if constexpr (!MV) ++a;
              break;
            }
          }
          if (tt < 0.0) lo = tt; else hi = tt;
        }
      }
      // a now counts the rejected shrink candidates in every form above
      if constexpr (MV) {
        if (tid == 0) {
          sStep[4 * sl + 0] = nprobe;
          sStep[4 * sl + 2] = a;
          sStep[4 * sl + 3] = accepted ? 1 : 0;
        }
      }
    }
  }
  __syncthreads();
  const int slot = R.dead[j];
  for (int i = tid; i < d; i += NT) R.u[(size_t)slot * d + i] = sX[i];
  if constexpr (MV) {
    fold(R.m - ((R.m - 1) / SL_CHUNK) * SL_CHUNK);   // the last chunk (wave 0 reads its own results below)
    // the chain's histogram into the iteration's record (zeroed by the
    // preparation kernel); integer sums, so the total is exact in any order
    if (tid < PROBE_HIST && t < (uint64_t)R.trace_cap && sCnt[tid] != 0)
      atomicAdd(&R.trace[t].hist[tid], sCnt[tid]);
    if (tid == 0) {
      R.nso[j] = sCnt[PROBE_HIST];
      R.nsh[j] = sCnt[PROBE_HIST + 1];
      R.acc[j] = sCnt[PROBE_HIST + 2];
    }
  }
  if (tid == 0) {
    R.lam[slot] = lx;
    R.probes[j] = nprobe;
    R.bins[j] = nbins;
  }
}

template <int NDET, int NT, int LK, bool LDS, bool MV = false>
__global__ __launch_bounds__(NT, 2) void k_slice(const ModelDev* __restrict__ Mp, Tables T, RBTables RB, RunDev R) {
  extern __shared__ double smem[];
  slice_body<NDET, NT, LK, LDS, MV>(*Mp, T, RB, R, blockIdx.x, smem);
}


// ------------------------------------------------------------- termination
__device__ void term_body(const RunDev& R) {
  __shared__ double sbuf[1024];
  DevState* S = R.state;
  if (S->done) return;
  const int n = R.n, tid = threadIdx.x;
  // the state, read once up front (thread 0 writes it back at the end, after
  // the metrics record, so no load waits behind those stores)
  const int it = S->iter, wl = S->walk_len;
  const double lstar = S->lstar, logX = S->logX, logZ = S->logZ;
  const long long n_dead = S->n_dead, n_evals = S->n_evals, n_bins = S->n_bin_terms;
  const bool slice = R.kernel == 0;
  const bool moves = !slice || R.move_counts;   // acc holds this iteration's values
  double m = NEG_INF;
  for (int i = tid; i < n; i += 1024) m = fmax(m, order_value(R.lam[i]));
  m = block_max<1024>(m, sbuf);
  double e = 0.0;                  // sum exp(lambda - max)
  for (int i = tid; i < n; i += 1024) e += exp(order_value(R.lam[i]) - m);
  // per-chain totals (evaluations, bins, accepted walk proposals or moved
  // slice steps, expansions, shrinks) and the fewest and most evaluations of
  // a chain.  Only thread 0 needs them and the exponential sum: each wave
  // reduces its own, then wave 0 combines the waves (the exponential sum
  // in wave order; the counts are integers below 2^53, exact in any order)
  constexpr int NW = 1024 / 64;
  const int lane = tid & 63, wv = tid >> 6;
  double c[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double x[2] = {0.0, -2147483647.0};   // most and (negated) fewest evaluations
#pragma unroll 1
  for (int j = tid; j < R.k; j += 1024) {
    const double p = (double)R.probes[j];
    c[0] += p;
    c[1] += (double)R.bins[j];
    if (moves) c[2] += (double)R.acc[j];
    if (slice && moves) {
      c[3] += (double)R.nso[j];
      c[4] += (double)R.nsh[j];
    }
    x[0] = fmax(x[0], p);
    x[1] = fmax(x[1], -p);
  }
  e = wave_sum(e);
#pragma unroll
  for (int q = 0; q < 5; ++q) c[q] = wave_sum(c[q]);
#pragma unroll
  for (int q = 0; q < 2; ++q) x[q] = wave_max(x[q]);
  __syncthreads();                 // every thread has read block_max's values
  if (lane == 0) {
    sbuf[wv] = e;
#pragma unroll
    for (int q = 0; q < 5; ++q) sbuf[(1 + q) * NW + wv] = c[q];
#pragma unroll
    for (int q = 0; q < 2; ++q) sbuf[(6 + q) * NW + wv] = x[q];
  }
  __syncthreads();
  double s = 0.0;
  if (wv == 0) {
#pragma unroll
    for (int w = 0; w < NW; ++w) s += sbuf[w];
#pragma unroll
    for (int q = 0; q < 5; ++q) c[q] = wave_sum(lane < NW ? sbuf[(1 + q) * NW + lane] : 0.0);
#pragma unroll
    for (int q = 0; q < 2; ++q) x[q] = wave_max(lane < NW ? sbuf[(6 + q) * NW + lane] : NEG_INF);
  }
  const double pmax = x[0], nmin = x[1];
  // (the record's histogram was summed by the chains themselves)
  const bool rec_on = it < R.trace_cap;
  const double pe = c[0], pb = c[1];
  if (tid == 0) {
    const double logz_live = logX + m + log(s / n);
    if (rec_on) {
      IterRec& rc = R.trace[it];
      rc.iter = it;
      rc.probes_min = (int)(-nmin);
      rc.probes_max = (int)pmax;
      rc.pad = 0;
      rc.lstar = lstar;
      rc.logX = logX;
      rc.logZ = logZ;
      rc.log_remaining = logz_live - logZ;
      rc.probes = (long long)pe;
      rc.steps = (long long)R.k * (slice ? R.m : wl);
      rc.accepted = moves ? (long long)c[2] : -1;
      rc.stepouts = moves ? (long long)c[3] : -1;
      rc.shrinks = moves ? (long long)c[4] : -1;
    }
    int done = 0;
    if (R.log_term > NEG_INF && logz_live - logZ < R.log_term) done = 1;
    if (n_dead + R.k > R.cap) done = 2;
    S->n_evals = n_evals + (long long)pe;
    S->n_bin_terms = n_bins + (long long)pb;
    if (R.kernel == 1) {
      // next chain length: walk_accept acceptances at this iteration's rate
      const long long acc = (long long)c[2], prop = (long long)R.k * wl;
      long long want = acc > 0 ? ((long long)R.walk_accept * prop + acc - 1) / acc : R.walk_max;
      S->walk_len = (int)(want < 1 ? 1 : (want > R.walk_max ? R.walk_max : want));
    }
    S->iter = it + 1;
    S->done = done;
  }
}

__global__ __launch_bounds__(1024) void k_term(RunDev R) { term_body(R); }


// ------------------------------------------------------- random-walk chains
// The alternative inner kernel (the random walk of bilby's sampler, paper
// Section 2, read as differential-evolution moves): chain j = blockIdx.x, one
// wavefront, makes the iteration's walk_len proposals y = x + gamma (u_a -
// u_b) from two distinct survivors a, b (gamma = 1 or 2.38 / sqrt(2 d), each
// with probability 1/2, times a factor uniform on [0.9, 1.1]; periodic
// coordinates wrap) and accepts y iff it lies
// in the unit cube and lambda(y) > L* (two survivors at one point give the
// current point itself: a null move, not evaluated).  Proposals are set up
// 64 at a time:
// lane i takes proposal s + i from the current point (its draws, its two
// survivors, its probe's source set-up into a record in LDS); the wave then
// evaluates them in order and, at the first acceptance, moves and sets up
// the next batch from the new point.  The proposals evaluated and counted
// are exactly those of the sequential chain.
constexpr int WK_DOUBLES_FIXED = 64 * SL_PSTRIDE + 64 + 16;   // records, Gaussian values, position

template <int NDET, int LK, bool LDS>
__global__ __launch_bounds__(64, 2) void k_walk(const ModelDev* __restrict__ Mp, Tables T, RBTables RB, RunDev R) {
  extern __shared__ double smem[];
  const ModelDev& M = *Mp;
  const DevState* S = R.state;
  if (S->done) return;
  const int lane = threadIdx.x, j = blockIdx.x, d = R.d;
  const uint64_t t = (uint64_t)S->iter;
  const double lstar = S->lstar;
  const int len = S->walk_len;
  const int ns = R.n - R.k;
  double* sP = smem;
  double* sG = sP + 64 * SL_PSTRIDE;
  double* sX = sG + 64;
  double* stab = sX + 16;
  TabView V{};
  if constexpr (lk_full(LK)) V = stage_tables<NDET, lk_mixed(LK)>(M, T, LDS, stab, lane, 64);
  RBTables RBv = RB;
  if constexpr (lk_rb(LK) && LDS) RBv = stage_rb<NDET, lk_mixed(LK)>(RB, stab, lane, 64);
  const int start = R.start[j];
  if (lane < d) sX[lane] = R.u[(size_t)start * d + lane];
  double lx = R.lam[start];
  const double g_de = 2.38 / sqrt(2.0 * d);
  int nprobe = 0, nacc = 0;
  long long nbins = 0;
  __syncthreads();
  ProbeRec* rec = reinterpret_cast<ProbeRec*>(sP + lane * SL_PSTRIDE);
  for (int s = 0; s < len;) {
    // ---- proposals s .. s+63 from the current point, one per lane
    const int sp = s + lane;
    double y[MAX_DIM];
    bool cin = false;
    if (sp < len) {
      const u64x4 b = philox(t, (uint64_t)j, (uint64_t)sp, purpose_word(P_WALK, 0), R.key0, R.key1);
      const int ia = (int)floor(unif53(b.x[0]) * (double)ns);
      int ib = (int)floor(unif53(b.x[1]) * (double)(ns - 1));
      ib += (ib >= ia) ? 1 : 0;
      const double g = (unif53(b.x[2]) < 0.5 ? 1.0 : g_de) * fma(0.2, unif53(b.x[3]), 0.9);
      const double* ua = R.u + (size_t)R.surv[ia] * d;
      const double* ub = R.u + (size_t)R.surv[ib] * d;
      cin = true;
      bool same = true;   // two survivors at one point: a null move, not evaluated
#pragma unroll
      for (int i = 0; i < MAX_DIM; ++i) {
        if (i < d) {
          const double df = ua[i] - ub[i];
          same = same && df == 0.0;
          y[i] = cube_coord(M.periodic, i, fma(g, df, sX[i]));
          cin = cin && (((M.periodic >> i) & 1u) || (y[i] >= 0.0 && y[i] <= 1.0));
        } else {
          y[i] = 0.0;
        }
      }
      cin = cin && !same;
      if (cin) {
        if (LK == LK_GAUSS) {
          sG[lane] = gauss_lambda(M, y);
        } else {
          const int ka = probe_intrinsic(M, y, rec);
          if constexpr (lk_full(LK)) {
#pragma unroll
            for (int dd = 0; dd < NDET; ++dd) rec->hk[dd] = ka > 0 ? V.hpre[(size_t)dd * V.hstride + ka - 1] : 0.0;
          }
          probe_extrinsic<NDET>(M, y, rec);
        }
      }
    }
    const unsigned long long mask = __ballot(cin);
    __syncthreads();
    // ---- the batch in order, until the first acceptance
    int i = 0;
    bool moved = false;
    for (; i < 64 && s + i < len; ++i) {
      if (!((mask >> i) & 1ull)) continue;
      double l;
      int terms;
      if constexpr (LK == LK_GAUSS) {
        l = sG[i];
        terms = 0;
      } else {
        const Probe pb = probe_from_rec<NDET>(*reinterpret_cast<const ProbeRec*>(sP + i * SL_PSTRIDE), lk_full(LK));
        if constexpr (lk_rb(LK)) {
          l = rb_wave<NDET, lk_mixed(LK)>(pb, RBv, M.n_bins, lane, &terms);
        } else {
          l = wave_sum(fullgrid_partial<NDET, lk_mixed(LK), true>(pb, V, lane, 64)) - 0.5 * pb.hh;
          terms = pb.k_act;
        }
      }
      ++nprobe;
      nbins += terms;
      if (l > lstar) {
        if (lane == i) {
#pragma unroll
          for (int q = 0; q < MAX_DIM; ++q)
            if (q < d) sX[q] = y[q];
        }
        lx = l;
        ++nacc;
        moved = true;
        break;
      }
    }
    s += moved ? i + 1 : i;
    __syncthreads();
  }
  const int slot = R.dead[j];
  if (lane < d) R.u[(size_t)slot * d + lane] = sX[lane];
  if (lane == 0) {
    R.lam[slot] = lx;
    R.probes[j] = nprobe;
    R.bins[j] = nbins;
    R.acc[j] = nacc;
  }
}

template <int NDET, int LK, bool LDS>
hipError_t launch_walk_t(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB, const RunDev& R,
                         hipStream_t st) {
  size_t tab = 0;
  if (LDS) tab = lk_rb(LK) ? rb_stage_doubles(RB.nb, NDET, lk_mixed(LK)) * sizeof(double)
                           : staged_table_bytes(M.k_lim, NDET, lk_mixed(LK));
  const size_t lds = WK_DOUBLES_FIXED * sizeof(double) + tab;
  hipLaunchKernelGGL((k_walk<NDET, LK, LDS>), dim3(R.k), dim3(64), lds, st, Md, T, RB, R);
  return hipGetLastError();
}

// Tables staged in LDS while a CU still holds four chains.
template <int NDET>
hipError_t launch_walk_det(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                           const RunDev& R, hipStream_t st) {
  const bool rb = M.likelihood == LK_RB;
  const size_t tab = rb ? rb_stage_doubles(RB.nb, NDET, M.mixed != 0) * sizeof(double)
                        : staged_table_bytes(M.k_lim, NDET, M.mixed != 0);
  const bool lds = WK_DOUBLES_FIXED * sizeof(double) + tab <= 40 * 1024;
  if (rb) {
    if (M.mixed) return lds ? launch_walk_t<NDET, LK_RB32, true>(M, Md, T, RB, R, st)
                            : launch_walk_t<NDET, LK_RB32, false>(M, Md, T, RB, R, st);
    return lds ? launch_walk_t<NDET, LK_RB, true>(M, Md, T, RB, R, st)
               : launch_walk_t<NDET, LK_RB, false>(M, Md, T, RB, R, st);
  }
  if (M.mixed) return lds ? launch_walk_t<NDET, LK_FULL32, true>(M, Md, T, RB, R, st)
                          : launch_walk_t<NDET, LK_FULL32, false>(M, Md, T, RB, R, st);
  return lds ? launch_walk_t<NDET, LK_FULL, true>(M, Md, T, RB, R, st)
             : launch_walk_t<NDET, LK_FULL, false>(M, Md, T, RB, R, st);
}


// ---------------------------------------------------------------- packed
// Serving: one launch per kernel covers every resident run.  Blocks are
// assigned to runs by prefix offsets (off[r] = first block of run r).
__device__ inline int packed_run_of(const int* __restrict__ off, int nr, int b) {
  int lo = 0, hi = nr - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_rank_packed(const PackedRun* __restrict__ runs,
                                                     const int* __restrict__ off, int nr) {
  const int r = packed_run_of(off, nr, blockIdx.x);
  const RunDev& R = runs[r].R;
  if (R.state->done) return;
  const int i = (blockIdx.x - off[r]) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= R.n) return;
  rank_element(R.lam, R.n, R.k, R.rank, R.dead, nullptr, i, lane);
}

__global__ __launch_bounds__(1024) void k_prep_packed(const PackedRun* __restrict__ runs) {
  prep_body(runs[blockIdx.x].R);
}

__global__ __launch_bounds__(1024) void k_term_packed(const PackedRun* __restrict__ runs) {
  term_body(runs[blockIdx.x].R);
}

template <int NT, int LK>
__global__ __launch_bounds__(NT, 2) void k_slice_packed(const PackedRun* __restrict__ runs, const int* __restrict__ off,
                                                     int nr) {
  extern __shared__ double smem[];
  const int r = packed_run_of(off, nr, blockIdx.x);
  const PackedRun& P = runs[r];
  const int j = blockIdx.x - off[r];
  switch (P.M->n_det) {
    case 1: slice_body<1, NT, LK, false>(*P.M, P.T, P.RB, P.R, j, smem); break;
    case 2: slice_body<2, NT, LK, false>(*P.M, P.T, P.RB, P.R, j, smem); break;
    default: slice_body<3, NT, LK, false>(*P.M, P.T, P.RB, P.R, j, smem); break;
  }
}

__global__ void k_gather_done(const PackedRun* __restrict__ runs, int nr, int* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nr) out[r] = runs[r].R.state->done;
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
  const double2 sc_ = sincos_cycles(fma(f, p.dt[det], psi));
  const double sn = sc_.x, cs = sc_.y;
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

// Equal-weight samples by systematic resampling (the equal-weight count of
// the paper's results table, Section 3).  Pass 1, one workgroup: the
// normalised weights p_q = exp(log w_q - log Z) of the weighted samples (dead
// points in death order, then the live points), their running sum cum[q]
// (each thread sums a contiguous chunk, the chunk totals are scanned across
// the workgroup), and the one uniform u0 of the RESAMPLE purpose.
__global__ __launch_bounds__(1024) void k_resample_cum(RunDev R, long long total, double logZ, double* cum,
                                                       double* u0) {
  __shared__ double sscan[1024];
  const long long nd = R.state->n_dead;
  const int tid = threadIdx.x;
  const double live_lw = R.state->logX - log((double)R.n) - logZ;
  const long long C = (total + 1023) / 1024;
  const long long qb = (long long)tid * C, qe = (qb + C < total) ? qb + C : total;
  auto weight = [&](long long q) {
    const double lw = q < nd ? R.dlogw[q] - logZ : order_value(R.lam[q - nd]) + live_lw;
    return exp(lw);
  };
  double cs = 0.0;
  for (long long q = qb; q < qe; ++q) cs += weight(q);
  double acc = block_inclusive_scan<1024, double>(cs, sscan) - cs;
  for (long long q = qb; q < qe; ++q) {
    acc += weight(q);
    cum[q] = acc;
  }
  if (tid == 0) {
    const u64x4 b = philox(0, 0, 0, purpose_word(P_RESAMPLE, 0), R.key0, R.key1);
    u0[0] = unif53(b.x[0]);
  }
}

// Pass 2, one thread per output m: the position (m + u0) / n_out of the total
// weight and the first sample whose running sum exceeds it (binary search;
// the last sample if none does, which only rounding can cause).
__global__ void k_resample_pick(const ModelDev* __restrict__ Mp, RunDev R, long long total, const double* cum,
                                const double* u0, long long n_out, int* idx, double* theta) {
  const ModelDev& M = *Mp;
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_out) return;
  const double pos = ((double)m + u0[0]) / (double)n_out * cum[total - 1];
  long long lo = 0, hi = total - 1;   // the answer lies in [lo, hi]
  while (lo < hi) {
    const long long mid = lo + (hi - lo) / 2;
    if (cum[mid] > pos) hi = mid; else lo = mid + 1;
  }
  idx[m] = (int)lo;
  if (theta) {
    const long long nd = R.state->n_dead;
    const int d = R.d;
    const double* u = lo < nd ? R.du + lo * d : R.u + (size_t)(lo - nd) * d;
    for (int i = 0; i < d; ++i)
      theta[m * d + i] = (M.likelihood == LK_GAUSS) ? u[i] : prior_plain(M.prior, i, u[i]);
  }
}

template <int NDET, int LK, bool LDS>
hipError_t launch_loglike_t(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                            const double* u, long n, double* out, int* terms, Probe* pbuf, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (LK != LK_GAUSS && pbuf) {
    if (M.model == 1)
      hipLaunchKernelGGL(k_probe_setup, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Md, T.hpre, u, n, pbuf,
                         terms);
    else
      hipLaunchKernelGGL((k_probe_setup2<NDET>), dim3((unsigned)((n + SETUP2_PROBES - 1) / SETUP2_PROBES)), dim3(256),
                         setup2_lds_bytes(), st, Md, T.hpre, u, n, pbuf, terms);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = LDS ? staged_table_bytes(M.k_lim, NDET, lk_mixed(LK)) : 0;
    long blocks = (n + 15) / 16;
    if (blocks > 256 * 2) blocks = 256 * 2;
    hipLaunchKernelGGL((k_probe_bins<NDET, LK, LDS>), dim3((unsigned)blocks), dim3(1024), lds, st, Md, T, pbuf, n,
                       out);
    return hipGetLastError();
  }
  const size_t lds = LDS ? staged_table_bytes(M.k_lim, NDET, lk_mixed(LK)) : 0;
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((k_loglike<NDET, LK, LDS>), dim3((unsigned)blocks), dim3(256), lds, st, Md, T, RB, u, n, out,
                     terms);
  return hipGetLastError();
}

template <int NDET, int NT, int LK, bool LDS, bool MV = false>
hipError_t launch_slice_t(const ModelDev* Md, const Tables& T, const RBTables& RB, const RunDev& R, size_t lds,
                          hipStream_t st) {
  hipLaunchKernelGGL((k_slice<NDET, NT, LK, LDS, MV>), dim3(R.k), dim3(NT), lds, st, Md, T, RB, R);
  return hipGetLastError();
}

template <int NDET, int NT, bool MV = false>
hipError_t launch_slice_nt(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                           const RunDev& R, const LaunchCfg& C, hipStream_t st) {
  if (M.likelihood == LK_RB) {
    if (M.mixed)
      return C.lds_tables ? launch_slice_t<NDET, NT, LK_RB32, true, MV>(Md, T, RB, R, C.lds_bytes, st)
                          : launch_slice_t<NDET, NT, LK_RB32, false, MV>(Md, T, RB, R, C.lds_bytes, st);
    return C.lds_tables ? launch_slice_t<NDET, NT, LK_RB, true, MV>(Md, T, RB, R, C.lds_bytes, st)
                        : launch_slice_t<NDET, NT, LK_RB, false, MV>(Md, T, RB, R, C.lds_bytes, st);
  }
  if (M.mixed) {
    if (C.lds_tables) return launch_slice_t<NDET, NT, LK_FULL32, true, MV>(Md, T, RB, R, C.lds_bytes, st);
    return launch_slice_t<NDET, NT, LK_FULL32, false, MV>(Md, T, RB, R, C.lds_bytes, st);
  }
  if (C.lds_tables) return launch_slice_t<NDET, NT, LK_FULL, true, MV>(Md, T, RB, R, C.lds_bytes, st);
  return launch_slice_t<NDET, NT, LK_FULL, false, MV>(Md, T, RB, R, C.lds_bytes, st);
}

template <int NDET>
hipError_t launch_slice_det(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                            const RunDev& R, const LaunchCfg& C, hipStream_t st) {
  switch (C.slice_threads) {
    case 64: return launch_slice_nt<NDET, 64>(M, Md, T, RB, R, C, st);
    case 128: return launch_slice_nt<NDET, 128>(M, Md, T, RB, R, C, st);
    default: return launch_slice_nt<NDET, 256>(M, Md, T, RB, R, C, st);
  }
}

size_t slice_lds_fixed(int nt, bool mv) { return slice_fixed_doubles(nt, mv) * sizeof(double); }

template <int NT>
hipError_t launch_slice_packed_nt(const PackedRun* runs, const int* slice_off, int nr, int slice_blocks, int lk,
                                  size_t slice_lds, hipStream_t st) {
  switch (lk) {
    case LK_FULL:
      hipLaunchKernelGGL((k_slice_packed<NT, LK_FULL>), dim3(slice_blocks), dim3(NT), slice_lds, st, runs, slice_off, nr);
      break;
    case LK_FULL32:
      hipLaunchKernelGGL((k_slice_packed<NT, LK_FULL32>), dim3(slice_blocks), dim3(NT), slice_lds, st, runs, slice_off,
                         nr);
      break;
    case LK_RB:
      hipLaunchKernelGGL((k_slice_packed<NT, LK_RB>), dim3(slice_blocks), dim3(NT), slice_lds, st, runs, slice_off, nr);
      break;
    default:
      hipLaunchKernelGGL((k_slice_packed<NT, LK_RB32>), dim3(slice_blocks), dim3(NT), slice_lds, st, runs, slice_off,
                         nr);
      break;
  }
  return hipGetLastError();
}

}  // namespace

// The chain-kernel launchers of each group (one source file each).
hipError_t launch_slice_d1(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                           const RunDev& R, const LaunchCfg& C, hipStream_t st);
hipError_t launch_slice_d2(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                           const RunDev& R, const LaunchCfg& C, hipStream_t st);
hipError_t launch_slice_d3(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                           const RunDev& R, const LaunchCfg& C, hipStream_t st);
// the move-counting chain kernels (64 threads per chain)
hipError_t launch_slice_mv_d1(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                              const RunDev& R, const LaunchCfg& C, hipStream_t st);
hipError_t launch_slice_mv_d2(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                              const RunDev& R, const LaunchCfg& C, hipStream_t st);
hipError_t launch_slice_mv_d3(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                              const RunDev& R, const LaunchCfg& C, hipStream_t st);
hipError_t launch_slice_packed64(const PackedRun* runs, const int* slice_off, int nr, int slice_blocks, int lk,
                                 size_t slice_lds, hipStream_t st);
hipError_t launch_slice_packed128(const PackedRun* runs, const int* slice_off, int nr, int slice_blocks, int lk,
                                  size_t slice_lds, hipStream_t st);
hipError_t launch_slice_packed256(const PackedRun* runs, const int* slice_off, int nr, int slice_blocks, int lk,
                                  size_t slice_lds, hipStream_t st);

}  // namespace ns
