// Device-side building blocks of libns (gfx950, wave64): counter-based RNG,
// the selection key, a double-precision sincos in cycles, prior transforms
// and the per-probe TaylorF2 coefficients.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ns {

constexpr int MAX_DIM = 12;
constexpr int MAX_DET = 3;
constexpr double PI = 3.14159265358979323846;
constexpr double TWO_PI = 6.28318530717958647692;
constexpr double TSUN_S = 4.925490947641267e-6;     // G Msun / c^3  (s)
constexpr double C_SI = 299792458.0;                 // m/s
constexpr double MPC_S = 3.0856775814913673e22 / 299792458.0;  // 1 Mpc / c  (s)
constexpr double EULER_GAMMA = 0.57721566490153286061;

// RNG purposes: the high 16 bits of the last Philox counter word.
enum Purpose : uint64_t { P_INIT = 1, P_PICK = 2, P_DIR = 3, P_WIDTH = 4, P_SHRINK = 5, P_RESAMPLE = 6, P_SIGMA = 7, P_WALK = 8 };

// ------------------------------------------------------------------ Philox
// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128-bit
// products with the key bumped by the Weyl constants between rounds.
struct u64x4 { uint64_t x[4]; };

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ inline u64x4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                        uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint64_t h0 = mulhi64(M0, c0), l0 = M0 * c0;
    uint64_t h1 = mulhi64(M1, c2), l1 = M1 * c2;
    uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
    c0 = n0; c1 = l1; c2 = n2; c3 = l0;
  }
  u64x4 o; o.x[0] = c0; o.x[1] = c1; o.x[2] = c2; o.x[3] = c3;
  return o;
}

__host__ __device__ inline double unif53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

__host__ __device__ inline uint64_t purpose_word(uint64_t purpose, uint64_t idx) { return (purpose << 48) | idx; }

// ------------------------------------------------------------ order key
// Order-preserving map of a double to uint64: NaN is ordered as -inf and
// -0 as +0, so ascending keys are ascending values.
__host__ __device__ inline uint64_t order_key(double v) {
  if (v != v) v = -__builtin_inf();
  if (v == 0.0) v = 0.0;
  uint64_t b = (uint64_t)__builtin_bit_cast(uint64_t, v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ULL);
}

__host__ __device__ inline double order_value(double v) {
  if (v != v) return -__builtin_inf();
  return v == 0.0 ? 0.0 : v;
}

// ---------------------------------------------------------- sincos (cycles)
// sin and cos of 2 pi p for p in cycles.  The argument is reduced exactly to
// r in [-1/2, 1/2]; Taylor series of 2 sin(pi r) and cos(pi r) (terms to
// r^21 and r^20, truncation below 2e-17) give the half angle, and the
// double-angle identities sin 2a = 2 sin a cos a, cos 2a = 1 - 2 sin^2 a
// the result: fused multiply-adds only, no quadrant branches.  Absolute error
// below 1.3e-15 over the whole cycle.
__device__ inline double2 sincos_cycles(double p) {
  const double r = p - rint(p);
  const double r2 = r * r;
  double sp = fma(r2, 0x1.2877020d52cf0p-30, -0x1.8a404211f9547p-25);
  sp = fma(sp, r2, 0x1.aaec32af93359p-20);
  sp = fma(sp, r2, -0x1.6fadb9f155744p-15);
  sp = fma(sp, r2, 0x1.e8f434d018d63p-11);
  sp = fma(sp, r2, -0x1.e3074fde8871fp-7);
  sp = fma(sp, r2, 0x1.50783487ee782p-3);
  sp = fma(sp, r2, -0x1.32d2cce62bd86p+0);
  sp = fma(sp, r2, 0x1.466bc6775aae2p+2);
  sp = fma(sp, r2, -0x1.4abbce625be53p+3);
  sp = fma(sp, r2, 0x1.921fb54442d18p+2);
  const double s2 = r * sp;                      // 2 sin(pi r)
  double cp = fma(r2, 0x1.ef6e308d6d1c4p-29, -0x1.2a0c591af8314p-23);
  cp = fma(cp, r2, 0x1.20c62c2f2d7f5p-18);
  cp = fma(cp, r2, -0x1.b6e24f44b128fp-14);
  cp = fma(cp, r2, 0x1.f9d38a3763cc3p-10);
  cp = fma(cp, r2, -0x1.a6d1f2a204a8cp-6);
  cp = fma(cp, r2, 0x1.e1f506891babbp-3);
  cp = fma(cp, r2, -0x1.55d3c7e3cbffap+0);
  cp = fma(cp, r2, 0x1.03c1f081b5ac4p+2);
  cp = fma(cp, r2, -0x1.3bd3cc9be45dep+2);
  const double c = fma(cp, r2, 1.0);            // cos(pi r)
  return make_double2(s2 * c, fma(-0.5 * s2, s2, 1.0));
}

// ----------------------------------------------------------------- problem
struct PriorDev {
  int kind[MAX_DIM];
  double lo[MAX_DIM], hi[MAX_DIM];
  double a[MAX_DIM], b[MAX_DIM];  // per kind: UNIFORM lo,(hi-lo); COS cos lo,(cos hi-cos lo);
                                  // SIN sin lo,(sin hi-sin lo); VOLUME lo^3,(hi^3-lo^3)
};

struct DetDev {
  double D[6];      // detector tensor (x x^T - y y^T)/2: xx, xy, xz, yy, yz, zz
  double r_c[3];    // vertex / c (s)
};

// Everything a probe needs from the problem (passed by value to kernels).
struct ModelDev {
  int model, likelihood, n_dim, n_det;
  int n_bins, k_lim;           // k_lim: bins that can be active anywhere in the prior box
  double f_lo, df, gmst;
  double inv_df;               // 1 / df
  double fixed_dist_s;         // TF2_4P distance (s)
  PriorDev prior;
  DetDev det[MAX_DET];
  double gauss_mu[MAX_DIM];
  double gauss_inv2s2, gauss_norm;   // 1/(2 s^2), -d/2 ln(2 pi s^2)
  int mixed;                   // float bulk arithmetic (double phase, setup and evidence)
  double dw_scale;             // power of two: the float data table holds dw * dw_scale
  unsigned periodic;           // bit i: unit-cube coordinate i wraps around (modulo 1)
};

// Coordinate i of a point on a slice line: taken modulo 1 when periodic.
__device__ inline double cube_coord(unsigned periodic, int i, double y) {
  return ((periodic >> i) & 1u) ? y - floor(y) : y;
}

// Physical quantities of one parameter point, reduced to what the strain needs.
struct Phys {
  double mc_msun, eta, beta, sigma, dist_s, tc, phic;
  double so5, so6, so7;           // spin-orbit phase terms above 1.5PN (model 3; else 0)
  double hp, hx;                  // (1 + cos^2 i)/2 and cos i
  double sra, cra, sdec, cdec;    // sin/cos of (RA - GMST) and of Dec
  double s2psi, c2psi;            // sin/cos of 2 psi
};

// Per-probe coefficients of the phase and response.  Phases are in cycles.
struct Probe {
  double x, lnx;          // x = (pi M)^(1/3): v_k = x f_k^(1/3), ln v_k = ln x + ln f_k / 3
  double pref;            // 3/(128 eta) x^-5 / (2 pi): multiplies f_k^(-5/3) * series
  double c2, c3, c4, c5, c5l, c6, c6l, c7;   // series coefficients (ln v parts split)
  double tc;              // 2 pi f t_c in cycles is f * tc
  double ph0;             // (-phi_c - pi/4) / (2 pi)
  double kre[MAX_DET], kim[MAX_DET];   // A K_det (A includes the distance)
  double dt[MAX_DET];     // arrival delay (s): cycles f * dt
  double hh;              // <h|h> summed over the detectors (from the prefix table)
  double f_isco;
  int k_act;              // active bins k < k_act
};

// Number of grid bins with f_k <= f_isco, where f_k = f_lo + k df is rounded
// as a product followed by a sum (no fused multiply-add); in [0, n_bins].
// inv_df only seeds the estimate, which the two loops then make exact.
__device__ inline int active_bins(double f_lo, double df, double inv_df, int n_bins, double f_isco) {
#pragma clang fp contract(off)
  if (!(f_isco >= f_lo)) return 0;
  double est = (f_isco - f_lo) * inv_df;
  int k = (est >= (double)n_bins) ? n_bins : (int)floor(est) + 1;
  if (k > n_bins) k = n_bins;
  while (k > 0 && f_lo + (double)(k - 1) * df > f_isco) --k;
  while (k < n_bins && f_lo + (double)k * df <= f_isco) ++k;
  return k;
}

__device__ inline double prior_plain(const PriorDev& P, int i, double u) {
  double a = P.a[i], b = P.b[i];
  switch (P.kind[i]) {
    case 1: return acos(fma(u, b, a));
    case 2: return asin(fma(u, b, a));
    case 3: return cbrt(fma(u, b, a));
    default: return fma(u, b, a);
  }
}

// Affine (uniform) transform of coordinate i.
__device__ inline double prior_affine(const PriorDev& P, int i, double u) { return fma(u, P.b[i], P.a[i]); }

// Spin-orbit phase terms of waveform model 3 above 1.5PN, linear in the
// aligned spins: so5 joins the 2.5PN coefficient (inside its 1 + 3 ln v),
// so6 the 3PN and so7 the 3.5PN coefficient; chi_s, chi_a are the symmetric
// and antisymmetric spins and delta = (m1 - m2)/M.
__device__ inline void spin_orbit_coefficients(double eta, double c1, double c2, double delta, double* so5,
                                               double* so6, double* so7) {
  const double e2 = eta * eta, e3 = e2 * eta;
  const double cs = 0.5 * (c1 + c2), ca = 0.5 * (c1 - c2);
  *so5 = (732985.0 / 2268.0 - 24260.0 / 81.0 * eta - 340.0 / 9.0 * e2) * cs + (732985.0 / 2268.0 + 140.0 / 9.0 * eta) * delta * ca;
  *so6 = PI * (2270.0 / 3.0 * delta * ca + (2270.0 / 3.0 - 520.0 * eta) * cs);
  *so7 = (-25150083775.0 / 3048192.0 + 10566655595.0 / 762048.0 * eta - 1042165.0 / 3024.0 * e2 + 5345.0 / 36.0 * e3) * cs +
         delta * (-25150083775.0 / 3048192.0 + 26804935.0 / 6048.0 * eta - 1985.0 / 48.0 * e2) * ca;
}

// Unit-cube point -> physical quantities.  The model fixes which prior kinds
// each coordinate may use (checked at run creation): uniform everywhere,
// uniform-in-volume for the distance, isotropic (COS) for theta_jn and (SIN)
// for the declination, whose cosine/sine then come straight from u.
__device__ inline void phys_from_u(const ModelDev& M, const double* u, Phys* s) {
  s->beta = 0.0; s->sigma = 0.0; s->hp = 1.0; s->hx = 0.0;
  s->so5 = 0.0; s->so6 = 0.0; s->so7 = 0.0;
  s->sra = 0; s->cra = 1; s->sdec = 0; s->cdec = 1; s->s2psi = 0; s->c2psi = 1;
  const PriorDev& P = M.prior;
  s->mc_msun = prior_affine(P, 0, u[0]);
  if (M.model == 1) {
    s->eta = prior_affine(P, 1, u[1]);
    s->tc = prior_affine(P, 2, u[2]);
    s->phic = prior_affine(P, 3, u[3]);
    s->dist_s = M.fixed_dist_s;
    return;
  }
  const double q = prior_affine(P, 1, u[1]);
  const double c1 = prior_affine(P, 2, u[2]);
  const double c2 = prior_affine(P, 3, u[3]);
  const double opq = 1.0 + q;
  s->eta = q / (opq * opq);
  const double m1 = 1.0 / opq, m2 = q / opq;
  s->beta = (c1 * (113.0 * m1 * m1 + 75.0 * s->eta) + c2 * (113.0 * m2 * m2 + 75.0 * s->eta)) * (1.0 / 12.0);
  s->sigma = 79.0 / 8.0 * s->eta * c1 * c2;
  if (M.model == 3) spin_orbit_coefficients(s->eta, c1, c2, m1 - m2, &s->so5, &s->so6, &s->so7);
  const double dv = prior_affine(P, 4, u[4]);
  s->dist_s = (P.kind[4] == 3 ? cbrt(dv) : dv) * MPC_S;
  const double ci = (P.kind[5] == 1) ? prior_affine(P, 5, u[5])
                                     : sincos_cycles(prior_affine(P, 5, u[5]) * (1.0 / TWO_PI)).y;
  s->hp = 0.5 * fma(ci, ci, 1.0);
  s->hx = ci;
  const double2 p2 = sincos_cycles(prior_affine(P, 6, u[6]) * (1.0 / PI));   // angle 2 psi
  s->s2psi = p2.x;
  s->c2psi = p2.y;
  const double2 ra = sincos_cycles((prior_affine(P, 7, u[7]) - M.gmst) * (1.0 / TWO_PI));
  s->sra = ra.x;
  s->cra = ra.y;
  if (P.kind[8] == 2) {
    s->sdec = prior_affine(P, 8, u[8]);
    s->cdec = sqrt(fmax(0.0, 1.0 - s->sdec * s->sdec));
  } else {
    const double2 de = sincos_cycles(prior_affine(P, 8, u[8]) * (1.0 / TWO_PI));
    s->sdec = de.x;
    s->cdec = de.y;
  }
  s->tc = prior_affine(P, 9, u[9]);
  s->phic = prior_affine(P, 10, u[10]);
}

// Physical parameter vector -> physical quantities (waveform generation and
// the heterodyne fiducial).
__device__ inline void phys_from_theta(const ModelDev& M, const double* th, Phys* s) {
  s->beta = 0.0; s->sigma = 0.0; s->hp = 1.0; s->hx = 0.0;
  s->so5 = 0.0; s->so6 = 0.0; s->so7 = 0.0;
  s->sra = 0; s->cra = 1; s->sdec = 0; s->cdec = 1; s->s2psi = 0; s->c2psi = 1;
  s->mc_msun = th[0];
  if (M.model == 1) {
    s->eta = th[1]; s->tc = th[2]; s->phic = th[3]; s->dist_s = M.fixed_dist_s;
    return;
  }
  double q = th[1], c1 = th[2], c2 = th[3];
  double opq = 1.0 + q;
  s->eta = q / (opq * opq);
  double m1 = 1.0 / opq, m2 = q / opq;
  s->beta = (c1 * (113.0 * m1 * m1 + 75.0 * s->eta) + c2 * (113.0 * m2 * m2 + 75.0 * s->eta)) / 12.0;
  s->sigma = 79.0 / 8.0 * s->eta * c1 * c2;
  if (M.model == 3) spin_orbit_coefficients(s->eta, c1, c2, m1 - m2, &s->so5, &s->so6, &s->so7);
  s->dist_s = th[4] * MPC_S;
  const double ci = sincos_cycles(th[5] / TWO_PI).y;
  s->hp = 0.5 * fma(ci, ci, 1.0);
  s->hx = ci;
  const double2 p2 = sincos_cycles(th[6] / PI);
  s->s2psi = p2.x;
  s->c2psi = p2.y;
  const double2 ra = sincos_cycles((th[7] - M.gmst) / TWO_PI);
  s->sra = ra.x;
  s->cra = ra.y;
  const double2 de = sincos_cycles(th[8] / TWO_PI);
  s->sdec = de.x;
  s->cdec = de.y;
  s->tc = th[9];
  s->phic = th[10];
}

// Coefficients of the 3.5PN TaylorF2 phase with leading-order aligned-spin
// terms (spin-orbit beta at 1.5PN, spin-spin sigma at 2PN) and the
// spin-orbit terms so5, so6, so7 above them (zero except in model 3):
//   Psi = 2 pi f t_c - phi_c - pi/4 + 3/(128 eta v^5) sum_k psi_k v^k,
// with ln v at 2.5PN and psi_6 containing -(6848/21) ln(4 v).
__device__ inline void pn_coefficients(double eta, double beta, double sigma, double so5, double so6, double so7,
                                       Probe* p) {
  double e2 = eta * eta, e3 = e2 * eta;
  p->c2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
  p->c3 = -16.0 * PI + 4.0 * beta;
  p->c4 = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * e2 - 10.0 * sigma;
  double a5 = PI * (38645.0 / 756.0 - 65.0 / 9.0 * eta) - so5;
  p->c5 = a5;
  p->c5l = 3.0 * a5;
  p->c6 = 11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * PI * PI - 6848.0 / 21.0 * EULER_GAMMA
          - 6848.0 / 21.0 * 1.3862943611198906
          + (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * PI * PI) * eta + 76055.0 / 1728.0 * e2
          - 127825.0 / 1296.0 * e3 + so6;
  p->c6l = -6848.0 / 21.0;
  p->c7 = PI * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * e2) + so7;
}

// Physical quantities -> probe coefficients: masses, amplitude
// sqrt(5/24) pi^(-2/3) Mc^(5/6) / D, f_ISCO, antenna patterns of each
// detector (long-wavelength response of an L-shaped interferometer) and
// geocentre-to-detector delays.
__device__ inline void probe_from_phys(const ModelDev& M, const Phys& s, const double* hpre, Probe* p) {
  double ln_mc = log(s.mc_msun * TSUN_S);
  double ln_pim = 1.1447298858494002 + ln_mc - 0.6 * log(s.eta);   // ln(pi M)
  p->lnx = ln_pim * (1.0 / 3.0);
  p->x = exp(p->lnx);
  p->pref = (3.0 / 128.0 / TWO_PI) / s.eta * exp(-5.0 * p->lnx);
  pn_coefficients(s.eta, s.beta, s.sigma, s.so5, s.so6, s.so7, p);
  p->tc = s.tc;
  p->ph0 = (-s.phic - 0.25 * PI) * (1.0 / TWO_PI);
  double x3 = p->x * p->x * p->x;                    // pi M
  p->f_isco = 1.0 / (14.696938456699069 * x3);      // 1 / (6^(3/2) pi M)
  p->k_act = active_bins(M.f_lo, M.df, M.inv_df, M.n_bins, p->f_isco);
  if (p->k_act > M.k_lim) p->k_act = M.k_lim;
  double amp = 0.21278751013966343 * exp(5.0 / 6.0 * ln_mc) / s.dist_s;
  const bool have_h = hpre != nullptr && p->k_act > 0;
  if (M.model == 1) {
    p->kre[0] = amp; p->kim[0] = 0.0; p->dt[0] = 0.0;
    p->hh = have_h ? amp * amp * hpre[p->k_act - 1] : 0.0;
    return;
  }
  double hh = 0.0;
  // wave-frame axes at psi = 0: a = (sin phi, -cos phi, 0), b = (-cos phi sin dec, -sin phi sin dec, cos dec);
  // e+ = cos 2psi (a a - b b) + sin 2psi (a b + b a), ex = -sin 2psi (a a - b b) + cos 2psi (a b + b a)
  double ax = s.sra, ay = -s.cra;
  double bx = -s.cra * s.sdec, by = -s.sra * s.sdec, bz = s.cdec;
  double nx = s.cdec * s.cra, ny = s.cdec * s.sra, nz = s.sdec;
#pragma unroll
  for (int d = 0; d < MAX_DET; ++d) {
    if (d >= M.n_det) break;
    const double* D = M.det[d].D;
    double dax = D[0] * ax + D[1] * ay;
    double day = D[1] * ax + D[3] * ay;
    double daz = D[2] * ax + D[4] * ay;
    double dbx = D[0] * bx + D[1] * by + D[2] * bz;
    double dby = D[1] * bx + D[3] * by + D[4] * bz;
    double dbz = D[2] * bx + D[4] * by + D[5] * bz;
    double aDa = ax * dax + ay * day;
    double bDb = bx * dbx + by * dby + bz * dbz;
    double aDb = ax * dbx + ay * dby;
    (void)daz;
    double fp0 = aDa - bDb, fx0 = 2.0 * aDb;
    double fp = s.c2psi * fp0 + s.s2psi * fx0;
    double fx = -s.s2psi * fp0 + s.c2psi * fx0;
    p->kre[d] = amp * fp * s.hp;       // K = F+ (1 + cos^2 i)/2 - i Fx cos i
    p->kim[d] = -amp * fx * s.hx;
    if (have_h) hh += (p->kre[d] * p->kre[d] + p->kim[d] * p->kim[d]) * hpre[(size_t)d * M.n_bins + p->k_act - 1];
    const double* r = M.det[d].r_c;
    p->dt[d] = -(r[0] * nx + r[1] * ny + r[2] * nz);
  }
  p->hh = hh;
}

__device__ inline void make_probe(const ModelDev& M, const double* hpre, const double* u, Probe* p) {
  Phys s;
  phys_from_u(M, u, &s);
  probe_from_phys(M, s, hpre, p);
}

// ---- probe set-up split over two threads (chain kernel) ---------------------
// A candidate's set-up divides into an intrinsic half (masses, spins, phase
// coefficients, f_ISCO, active bins, the mass factor of the amplitude) and an
// extrinsic half (distance, inclination, antenna patterns, delays), which
// two threads compute side by side.  The halves meet in a ProbeRec; the
// evaluating threads assemble the Probe from it.
struct ProbeRec {
  double x, lnx, pref, c2, c3, c4, c5, c5l, c6, c6l, c7, tc, ph0;   // intrinsic
  double amp_mc;                    // sqrt(5/24) pi^(-2/3) Mc^(5/6) (intrinsic)
  double f_isco;                    // intrinsic
  int k_act, pad;                   // intrinsic
  double hk[MAX_DET];               // prefix-table entries at bin k_act - 1 (intrinsic; 0 if none)
  double inv_dist;                  // 1 / D (extrinsic)
  double gre[MAX_DET], gim[MAX_DET];   // F+ (1 + cos^2 i)/2 and -Fx cos i (extrinsic)
  double dt[MAX_DET];               // arrival delays (extrinsic)
};

// Both halves read every model constant they need before their first
// branch, and choose between the models with selects, so that the constant
// loads issue together instead of one round trip per use.
__device__ inline int probe_intrinsic(const ModelDev& M, const double* u, ProbeRec* r) {
  const PriorDev& P = M.prior;
  const bool m4p = M.model == 1;
  const double f_lo = M.f_lo, df = M.df, inv_df = M.inv_df;
  const int n_bins = M.n_bins, k_lim = M.k_lim;
  const double mc_msun = prior_affine(P, 0, u[0]);
  const double v1 = prior_affine(P, 1, u[1]), v2 = prior_affine(P, 2, u[2]), v3 = prior_affine(P, 3, u[3]);
  const double v9 = prior_affine(P, 9, u[9]), v10 = prior_affine(P, 10, u[10]);
  // TF2_4P: (Mc, eta, t_c, phi_c); TF2_11P: (Mc, q, chi1, chi2, ..., t_c, phi_c)
  const double q = v1, c1 = v2, c2 = v3;
  const double m1 = 1.0 / (1.0 + q), m2 = q * m1;   // component masses over M
  const double eta_q = m1 * m2;
  const double beta_q = (c1 * (113.0 * m1 * m1 + 75.0 * eta_q) + c2 * (113.0 * m2 * m2 + 75.0 * eta_q)) * (1.0 / 12.0);
  const double sigma_q = 79.0 / 8.0 * eta_q * c1 * c2;
  const double eta = m4p ? v1 : eta_q;
  const double beta = m4p ? 0.0 : beta_q;
  const double sigma = m4p ? 0.0 : sigma_q;
  double so5 = 0.0, so6 = 0.0, so7 = 0.0;
  if (M.model == 3) spin_orbit_coefficients(eta_q, c1, c2, m1 - m2, &so5, &so6, &so7);
  const double tc = m4p ? v2 : v9;
  const double phic = m4p ? v3 : v10;
  const double ln_mc = log(mc_msun * TSUN_S);
  const double ln_pim = 1.1447298858494002 + ln_mc - 0.6 * log(eta);   // ln(pi M)
  Probe p;
  p.lnx = ln_pim * (1.0 / 3.0);
  p.x = exp(p.lnx);
  const double x2 = p.x * p.x;
  p.pref = (3.0 / 128.0 / TWO_PI) / (eta * (x2 * x2 * p.x));
  pn_coefficients(eta, beta, sigma, so5, so6, so7, &p);
  r->x = p.x; r->lnx = p.lnx; r->pref = p.pref;
  r->c2 = p.c2; r->c3 = p.c3; r->c4 = p.c4; r->c5 = p.c5; r->c5l = p.c5l; r->c6 = p.c6; r->c6l = p.c6l; r->c7 = p.c7;
  r->tc = tc;
  r->ph0 = (-phic - 0.25 * PI) * (1.0 / TWO_PI);
  const double x3 = p.x * p.x * p.x;                 // pi M
  r->f_isco = 1.0 / (14.696938456699069 * x3);      // 1 / (6^(3/2) pi M)
  int k = active_bins(f_lo, df, inv_df, n_bins, r->f_isco);
  k = k > k_lim ? k_lim : k;
  r->k_act = k;
  // sqrt(5/24) pi^(-2/3) Mc^(5/6) with Mc^(5/6) = pi^(-5/6) (pi M)^(5/6) eta^(1/2)
  // = pi^(-5/6) x^(5/2) eta^(1/2): one square root instead of an exponential
  r->amp_mc = 0.08196993152115736 * (x2 * sqrt(p.x * eta));   // sqrt(5/24) pi^(-3/2)
  return k;
}

template <int NDET>
__device__ inline void probe_extrinsic(const ModelDev& M, const double* u, ProbeRec* r) {
  const PriorDev& P = M.prior;
  const bool m4p = M.model == 1;
  const double fixed_dist_s = M.fixed_dist_s, gmst = M.gmst;
  const int k4 = P.kind[4], k5 = P.kind[5], k8 = P.kind[8];
  const double dv = prior_affine(P, 4, u[4]), v5 = prior_affine(P, 5, u[5]), v6 = prior_affine(P, 6, u[6]);
  const double v7 = prior_affine(P, 7, u[7]), v8 = prior_affine(P, 8, u[8]);
  if (m4p) {
    r->inv_dist = 1.0 / fixed_dist_s;
    r->gre[0] = 1.0; r->gim[0] = 0.0; r->dt[0] = 0.0;
    return;
  }
  r->inv_dist = 1.0 / ((k4 == 3 ? cbrt(dv) : dv) * MPC_S);
  const double ci = (k5 == 1) ? v5 : sincos_cycles(v5 * (1.0 / TWO_PI)).y;
  const double hp = 0.5 * fma(ci, ci, 1.0), hx = ci;
  const double2 p2 = sincos_cycles(v6 * (1.0 / PI));   // angle 2 psi
  const double2 ra = sincos_cycles((v7 - gmst) * (1.0 / TWO_PI));
  double sdec, cdec;
  if (k8 == 2) {
    sdec = v8;
    cdec = sqrt(fmax(0.0, 1.0 - sdec * sdec));
  } else {
    const double2 de = sincos_cycles(v8 * (1.0 / TWO_PI));
    sdec = de.x;
    cdec = de.y;
  }
  // wave-frame axes at psi = 0 (see probe_from_phys)
  const double ax = ra.x, ay = -ra.y;
  const double bx = -ra.y * sdec, by = -ra.x * sdec, bz = cdec;
  const double nx = cdec * ra.y, ny = cdec * ra.x, nz = sdec;
#pragma unroll
  for (int d = 0; d < NDET; ++d) {
    const double* D = M.det[d].D;
    const double dax = D[0] * ax + D[1] * ay;
    const double day = D[1] * ax + D[3] * ay;
    const double dbx = D[0] * bx + D[1] * by + D[2] * bz;
    const double dby = D[1] * bx + D[3] * by + D[4] * bz;
    const double dbz = D[2] * bx + D[4] * by + D[5] * bz;
    const double aDa = ax * dax + ay * day;
    const double bDb = bx * dbx + by * dby + bz * dbz;
    const double aDb = ax * dbx + ay * dby;
    const double fp0 = aDa - bDb, fx0 = 2.0 * aDb;
    const double fp = p2.y * fp0 + p2.x * fx0;
    const double fx = -p2.x * fp0 + p2.y * fx0;
    r->gre[d] = fp * hp;
    r->gim[d] = -fx * hx;
    const double* rc = M.det[d].r_c;
    r->dt[d] = -(rc[0] * nx + rc[1] * ny + rc[2] * nz);
  }
}

// The Probe of a record; with_hh: <h|h> from the record's prefix-table
// entries (else 0).
template <int NDET>
__device__ inline Probe probe_from_rec(const ProbeRec& r, bool with_hh) {
  Probe p;
  p.x = r.x; p.lnx = r.lnx; p.pref = r.pref;
  p.c2 = r.c2; p.c3 = r.c3; p.c4 = r.c4; p.c5 = r.c5; p.c5l = r.c5l; p.c6 = r.c6; p.c6l = r.c6l; p.c7 = r.c7;
  p.tc = r.tc; p.ph0 = r.ph0; p.f_isco = r.f_isco; p.k_act = r.k_act;
  const double amp = r.amp_mc * r.inv_dist;
  double hh = 0.0;
#pragma unroll
  for (int d = 0; d < NDET; ++d) {
    p.kre[d] = amp * r.gre[d];
    p.kim[d] = amp * r.gim[d];
    p.dt[d] = r.dt[d];
    if (with_hh && r.k_act > 0) hh += (p.kre[d] * p.kre[d] + p.kim[d] * p.kim[d]) * r.hk[d];
  }
  p.hh = hh;
  return p;
}

// Phase of bin k in cycles (without the detector delay).
__device__ inline double phase_cycles(const Probe& p, double f, double f13, double lnf3, double fm53) {
  double v = p.x * f13;
  double lnv = p.lnx + lnf3;
  double s = fma(v, p.c7, fma(p.c6l, lnv, p.c6));
  s = fma(v, s, fma(p.c5l, lnv, p.c5));
  s = fma(v, s, p.c4);
  s = fma(v, s, p.c3);
  s = fma(v, s, p.c2);
  s = fma(v * v, s, 1.0);
  return fma(f, p.tc, p.ph0) + p.pref * fm53 * s;
}

}  // namespace ns
