// Device-side building blocks shared by the library's HIP sources:
// constants, the per-proposal prologue (TaylorF2 coefficients, antenna
// patterns, delays, amplitudes), FP64 sin/cos in cycles, ln I0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gw_i0_fit.h"

namespace gw {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kTwoPi = 6.283185307179586476925286766559005768;
constexpr double kInvTwoPi = 0.159154943091895335768883763372514362;
constexpr double kLog2E = 1.44269504088896340735992468100189214;
constexpr double kMsunSec = 4.925490947641267e-6;     // G Msun / c^3 (s)
constexpr double kLightSpeed = 299792458.0;            // m / s
constexpr double kMpcMetre = 3.085677581491367e22;     // m
constexpr double kEulerGamma = 0.5772156649015328606;
constexpr double kLog4 = 1.386294361119890618834464242916;

constexpr int kMaxDet = 4;

// Column indices of the per-proposal coefficient table (structure of arrays,
// column c of a batch of n lives at coef[c * n + p]).
enum CoefCol {
  // phase in cycles: psi(f) = xm5 * P(x) + (b5 + b6 x) ln f, x = f^(1/3),
  // P(x) = a0 + a2 x^2 + ... + a8 x^8 + a10 x^10 + a12 x^12, with the
  // linear-in-f time shift of detector 0 in a8 and the constant phase in a5.
  C_A0 = 0, C_A2, C_A3, C_A4, C_A5, C_A6, C_A7, C_A8, C_A10, C_A12, C_B5, C_B6,
  C_DT1 = 12,        // t-shift of detector i (i >= 1) relative to detector 0, s
  C_VALID = 15,      // 1 for a physical row, 0 otherwise
  C_APRE = 16,       // Re(A P_i), i < kMaxDet
  C_APIM = 20,       // Im(A P_i)
  C_HH = 24,         // <h|h> summed over detectors (closed form)
  C_TAU0 = 25,       // total time shift of detector 0 (t_c + dt_0), s
  C_AMP = 26,        // amplitude A
  C_NCOEF = 32
};

// Detector network and grid constants passed by value to kernels.
struct Geom {
  double tensor[kMaxDet][9];
  double pos[kMaxDet][3];
  double hhw[kMaxDet];   // W_i = 4 df sum_k f_k^(-7/3) / S_ik
  double gmst;
  double df;
  int64_t k0;
  int64_t n_freq;
  int32_t n_det;
};

__device__ inline bool finite_d(double v) { return __builtin_isfinite(v); }

// Per-proposal prologue.  Writes C_NCOEF values into out[] (stride ``ld``).
// marg: 0 plain, 1 phase-marginalised (phi_c := 0), 2 phase+distance
// (phi_c := 0, d_L := 1 Mpc), 3 phase+time (phi_c := 0, t_c := 0).
__device__ inline void prologue(const double* __restrict__ th, int marg, const Geom& g,
                                double* out, int64_t ld) {
  double v[13];
#pragma unroll
  for (int j = 0; j < 13; ++j) v[j] = th[j];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 13; ++j) ok = ok && finite_d(v[j]);
  const double mc = v[0], q = v[1], c1 = v[2], c2 = v[3], l1 = v[4], l2 = v[5];
  double dl = v[6];
  const double iota = v[7], ra = v[8], dec = v[9], psi = v[10];
  double phic = v[11];
  double tc = v[12];
  ok = ok && mc > 0.0 && q > 0.0 && q <= 1.0 && fabs(c1) < 1.0 && fabs(c2) < 1.0;
  if (marg != 2) ok = ok && dl > 0.0;
  if (!ok) {
#pragma unroll
    for (int c = 0; c < C_NCOEF; ++c) out[c * ld] = 0.0;
    return;
  }
  if (marg != 0) phic = 0.0;
  if (marg == 2) dl = 1.0;
  if (marg == 3) tc = 0.0;

  // Masses: X1 = m1/M >= X2, eta = X1 X2, delta = X1 - X2.
  const double x1 = 1.0 / (1.0 + q);
  const double x2 = q * x1;
  const double eta = x1 * x2;
  const double dlt = x1 - x2;
  const double mtot = mc * pow(eta, -0.6);
  const double eta2 = eta * eta, eta3 = eta2 * eta;

  // Aligned-spin combinations.
  const double sl = x1 * x1 * c1 + x2 * x2 * c2;
  const double dsl = dlt * (x2 * c2 - x1 * c1);

  // Post-Newtonian coefficients of sum_j (p_j + l_j ln v) v^j.
  const double p0 = 1.0;
  const double p2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
  const double p3 = -16.0 * kPi + 188.0 / 3.0 * sl + 25.0 * dsl;
  const double sig = 79.0 / 8.0 * eta * c1 * c2 + 81.0 / 16.0 * (x1 * x1 * c1 * c1 + x2 * x2 * c2 * c2);
  const double p4 = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * eta2 - 10.0 * sig;
  const double gam = (554345.0 / 1134.0 + 110.0 / 9.0 * eta) * sl + (13915.0 / 84.0 - 10.0 / 3.0 * eta) * dsl;
  const double p5 = kPi * (38645.0 / 756.0 - 65.0 / 9.0 * eta) - gam;
  const double l5 = 3.0 * p5;
  const double p6 = 11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * kPi * kPi
                    - 6848.0 / 21.0 * (kEulerGamma + kLog4)
                    + (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * kPi * kPi) * eta
                    + 76055.0 / 1728.0 * eta2 - 127825.0 / 1296.0 * eta3
                    + kPi * (3760.0 * sl + 1490.0 * dsl) / 3.0;
  const double l6 = -6848.0 / 21.0;
  const double p7 = kPi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * eta2)
                    + (-8980424995.0 / 762048.0 + 6586595.0 / 756.0 * eta - 305.0 / 36.0 * eta2) * sl
                    - (170978035.0 / 48384.0 - 2876425.0 / 672.0 * eta - 4735.0 / 144.0 * eta2) * dsl;
  // Tidal (Lambda-tilde at 5PN, delta-Lambda-tilde at 6PN).
  const double lp = l1 + l2, lm = l1 - l2;
  const double ltil = 8.0 / 13.0 * ((1.0 + 7.0 * eta - 31.0 * eta2) * lp + dlt * (1.0 + 9.0 * eta - 11.0 * eta2) * lm);
  const double dltil = 0.5 * (dlt * (1.0 - 13272.0 / 1319.0 * eta + 8944.0 / 1319.0 * eta2) * lp
                              + (1.0 - 15910.0 / 1319.0 * eta + 32850.0 / 1319.0 * eta2 + 3380.0 / 1319.0 * eta3) * lm);
  const double t10 = -19.5 * ltil;
  const double t12 = -3115.0 / 64.0 * ltil + 6595.0 / 364.0 * dlt * dltil;

  // v = kappa x with kappa = (pi M)^(1/3), x = f^(1/3); ln v = ln kappa + ln f / 3.
  const double kap = cbrt(kPi * mtot * kMsunSec);
  const double lk = log(kap);
  const double ki = 1.0 / kap;
  const double ki2 = ki * ki, ki3 = ki2 * ki, ki5 = ki3 * ki2;
  const double pref = 3.0 / (128.0 * eta) * kInvTwoPi;  // cycles
  double a[13];
  a[0] = pref * ki5 * p0;
  a[2] = pref * ki3 * p2;
  a[3] = pref * ki2 * p3;
  a[4] = pref * ki * p4;
  a[5] = pref * (p5 + l5 * lk) + (-phic - 0.25 * kPi) * kInvTwoPi;
  a[6] = pref * kap * (p6 + l6 * lk);
  a[7] = pref * kap * kap * p7;
  const double kap5 = kap * kap * kap * kap * kap;
  a[10] = pref * kap5 * t10;
  a[12] = pref * kap5 * kap * kap * t12;
  const double b5 = pref * l5 / 3.0;
  const double b6 = pref * l6 * kap / 3.0;

  // Detector frame: phi = ra - gmst.
  const double ph = ra - g.gmst;
  double sp, cp, sd, cd, ss, cs;
  sincos(ph, &sp, &cp);
  sincos(dec, &sd, &cd);
  sincos(psi, &ss, &cs);
  const double s[3] = {cd * cp, cd * sp, sd};
  const double m[3] = {-sp, cp, 0.0};
  const double nn[3] = {-sd * cp, -sd * sp, cd};
  double X[3], Y[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    X[j] = -cs * m[j] + ss * nn[j];
    Y[j] = ss * m[j] + cs * nn[j];
  }
  const double amp = sqrt(5.0 / 24.0) * pow(kPi, -2.0 / 3.0) * kLightSpeed / (dl * kMpcMetre)
                     * pow(mc * kMsunSec, 5.0 / 6.0);
  const double ci = cos(iota);
  const double pp = 0.5 * (1.0 + ci * ci);
  double tau0 = 0.0, hh = 0.0;
#pragma unroll
  for (int i = 0; i < kMaxDet; ++i) {
    double fp = 0.0, fx = 0.0, dt = 0.0;
    if (i < g.n_det) {
      const double* D = g.tensor[i];
      double DX[3], DY[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        DX[r] = D[3 * r] * X[0] + D[3 * r + 1] * X[1] + D[3 * r + 2] * X[2];
        DY[r] = D[3 * r] * Y[0] + D[3 * r + 1] * Y[1] + D[3 * r + 2] * Y[2];
      }
      fp = (X[0] * DX[0] + X[1] * DX[1] + X[2] * DX[2]) - (Y[0] * DY[0] + Y[1] * DY[1] + Y[2] * DY[2]);
      fx = (X[0] * DY[0] + X[1] * DY[1] + X[2] * DY[2]) + (Y[0] * DX[0] + Y[1] * DX[1] + Y[2] * DX[2]);
      dt = -(s[0] * g.pos[i][0] + s[1] * g.pos[i][1] + s[2] * g.pos[i][2]) / kLightSpeed;
    }
    const double tau = tc + dt;
    if (i == 0) tau0 = tau;
    const double apr = amp * fp * pp;
    const double api = -amp * fx * ci;
    out[(C_APRE + i) * ld] = apr;
    out[(C_APIM + i) * ld] = api;
    if (i >= 1 && i < 4) out[(C_DT1 + i - 1) * ld] = (i < g.n_det) ? tau - tau0 : 0.0;
    if (i < g.n_det) hh += (apr * apr + api * api) * g.hhw[i];
  }
  a[8] = tau0;
  out[C_A0 * ld] = a[0];
  out[C_A2 * ld] = a[2];
  out[C_A3 * ld] = a[3];
  out[C_A4 * ld] = a[4];
  out[C_A5 * ld] = a[5];
  out[C_A6 * ld] = a[6];
  out[C_A7 * ld] = a[7];
  out[C_A8 * ld] = a[8];
  out[C_A10 * ld] = a[10];
  out[C_A12 * ld] = a[12];
  out[C_B5 * ld] = b5;
  out[C_B6 * ld] = b6;
  out[C_VALID * ld] = 1.0;
  out[C_HH * ld] = hh;
  out[C_TAU0 * ld] = tau0;
  out[C_AMP * ld] = amp;
#pragma unroll
  for (int c = C_AMP + 1; c < C_NCOEF; ++c) out[c * ld] = 0.0;
}

// Phase in cycles of the template at one frequency, from the coefficient
// registers: xm5 * P(x) + (b5 + b6 x) ln f.
struct PhaseCoef {
  double a0, a2, a3, a4, a5, a6, a7, a8, a10, a12, b5, b6;
};

__device__ inline double phase_cycles(const PhaseCoef& c, double x, double x2, double xm5, double lnf) {
  double t = fma(x2, c.a12, c.a10);
  t = fma(x2, t, c.a8);
  t = fma(x, t, c.a7);
  t = fma(x, t, c.a6);
  t = fma(x, t, c.a5);
  t = fma(x, t, c.a4);
  t = fma(x, t, c.a3);
  t = fma(x, t, c.a2);
  t = fma(x2, t, c.a0);
  const double lg = fma(c.b6, x, c.b5);
  return fma(lg, lnf, t * xm5);
}

// Coefficients of the FP64 sin/cos polynomials.  Kernels take them as a
// kernel argument so that they sit in SGPRs (a VOP3 FMA can read one SGPR
// pair directly, which avoids a register copy per coefficient).
struct TrigConsts {
  double s[10];  // sin: (-1)^j / (2j+3)!, j = 0..9  (a^3 .. a^21)
  double c[11];  // cos: (-1)^(j+1) / (2j+2)!, j = 0..10 (a^2 .. a^22)
};

__host__ __device__ inline TrigConsts make_trig_consts() {
  TrigConsts t;
  double fact = 1.0;  // n!
  int n = 1;
  for (int j = 0; j < 10; ++j) {
    while (n < 2 * j + 3) fact *= (double)(++n);
    t.s[j] = ((j & 1) ? 1.0 : -1.0) / fact;
  }
  fact = 1.0;
  n = 1;
  for (int j = 0; j < 11; ++j) {
    while (n < 2 * j + 2) fact *= (double)(++n);
    t.c[j] = ((j & 1) ? 1.0 : -1.0) / fact;
  }
  return t;
}

// sin and cos of 2 pi r for a phase r in cycles, FP64.  The phase is reduced
// to the nearest half turn (exact in FP64: r * 2 and r - q / 2 are exact), the
// remainder |a| <= pi/2 rad goes through the Taylor series of sin to a^21 and
// of cos to a^22 (truncation below 2e-18 on that interval), and the half-turn
// count flips both signs.
__device__ inline void sincos_cycles(double r, const TrigConsts& T, double* s_out, double* c_out) {
  const double q = rint(r * 2.0);
  const double t = fma(q, -0.5, r);
  const double a = t * kTwoPi;
  const double a2 = a * a;
  double ps = T.s[9];
#pragma unroll
  for (int j = 8; j >= 0; --j) ps = fma(ps, a2, T.s[j]);
  const double sn = fma(a * a2, ps, a);
  double pc = T.c[10];
#pragma unroll
  for (int j = 9; j >= 0; --j) pc = fma(pc, a2, T.c[j]);
  const double cn = fma(a2, pc, 1.0);
  // (-1)^q on both: flip the sign bits when q is odd.
  const unsigned flip = ((unsigned)(int)q) << 31;
  *s_out = __hiloint2double(__double2hiint(sn) ^ flip, __double2loint(sn));
  *c_out = __hiloint2double(__double2hiint(cn) ^ flip, __double2loint(cn));
}

// ln I0(x), x >= 0, at a fixed cost.  For x < 20 the defining power series
// I0(x) = sum_k (x^2/4)^k / (k!)^2, summed by Horner in y = x^2/4 with 40
// terms (truncation below 1e-23 relative on that range); for x >= 20 the
// large-argument expansion I0(x) ~ e^x / sqrt(2 pi x) sum_k c_k x^-k with
// c_k = ((2k-1)!!)^2 / (k! 8^k) (Abramowitz & Stegun 9.7.1), Horner in
// u = 1/x with 24 terms (the terms still decrease there; truncation below
// 1e-16).  The coefficients are fixed at compile time (below).
struct I0Coefs {
  double ser[40];
  double asy[24];
};

constexpr I0Coefs make_i0_coefs() {
  I0Coefs c{};
  double f = 1.0;
  for (int k = 0; k < 40; ++k) {
    if (k > 0) f *= (double)k;
    c.ser[k] = 1.0 / (f * f);
  }
  double a = 1.0;
  for (int k = 0; k < 24; ++k) {
    if (k > 0) a *= (double)(2 * k - 1) * (double)(2 * k - 1) / (8.0 * k);
    c.asy[k] = a;
  }
  return c;
}

constexpr I0Coefs kI0 = make_i0_coefs();

// Per-context constants of the distance marginal (kernels take them by
// device pointer).
struct LogI0Consts {
  double r1max;  // largest 1/d of the distance grid (bounds x = |Z1| / d); 0 if unknown
  double dmax;   // largest d of the grid (bounds u = 1/x = d / |Z1|); 0 if unknown
  double exp2_64[64];  // 2^(i/64), i < 64, rounded to FP64 (for exp_nonpos)
};

// The host fills exp2_64 from long-double 2^(i/64).
inline LogI0Consts make_log_i0_consts() {
  LogI0Consts c;
  c.r1max = 0.0;
  c.dmax = 0.0;
  for (int i = 0; i < 64; ++i) c.exp2_64[i] = (double)exp2l((long double)i / 64.0L);
  return c;
}

// exp(e) for -700 < e <= 0 (the distance marginal's terms relative to their
// bound), by the table method: e = (64 n + i) ln2/64 + r with |r| <= ln2/128
// (ln2/64 split in two parts so that k ln2/64 is exact for |k| < 2^13, i.e.
// e > -88; beyond that the reduction loses digits of terms below e^-88),
// exp(r) by its Taylor polynomial to r^5 (the first dropped term is below
// 4e-17), and exp(e) = 2^n 2^(i/64) exp(r).
__device__ inline double exp_nonpos(double e, const double* __restrict__ t64) {
  constexpr double kInvStep = 0x1.71547652b82fep+6;   // 64 / ln 2
  constexpr double kStepHi = 0x1.62e42fefa4000p-7;    // ln 2 / 64, leading 40 bits
  constexpr double kStepLo = -0x1.8432a1b0e2634p-49;  // ln 2 / 64 - kStepHi
  const double k = rint(e * kInvStep);
  const double r = fma(-k, kStepLo, fma(-k, kStepHi, e));
  const int ki = (int)k;
  double p = 1.0 / 120.0;
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(t64[ki & 63] * p, ki >> 6);
}

// The coefficients in constant memory, read with scalar loads where they are
// used: the empty asm on the table's address keeps the compiler from hoisting
// the 64 values out of the distance loops (they exceed the scalar registers,
// and hoisted into vector registers each Horner step costs extra moves), and
// sgpr() keeps each value in the scalar register the load wrote, so that a
// Horner step is one multiply-add with a scalar operand.  Materialising the
// constants with scalar moves instead costs two scalar instructions per use,
// as many as the vector work of the loops.
static __constant__ I0Coefs kI0Dev = make_i0_coefs();

typedef const __attribute__((address_space(4))) double* I0Table;

__device__ inline I0Table i0_table() {
  I0Table p = (I0Table)&kI0Dev.ser[0];
  asm volatile("" : "+s"(p));
  return p;
}

__device__ inline double sgpr(double c) {
  asm volatile("" : "+s"(c));
  return c;
}

// Power series of I0 in y = x^2 / 4 truncated after K terms (Horner).
template <int K>
__device__ inline double i0_series(double y) {
  const I0Table t = i0_table();
  double p = sgpr(t[K - 1]);
#pragma unroll
  for (int k = K - 2; k >= 0; --k) p = fma(p, y, sgpr(t[k]));
  return p;
}

// Large-argument series sum_k c_k u^k truncated after K terms (Horner).
template <int K>
__device__ inline double i0_asym_k(double u) {
  const I0Table t = i0_table() + 40;
  double p = sgpr(t[K - 1]);
#pragma unroll
  for (int k = K - 2; k >= 0; --k) p = fma(p, u, sgpr(t[k]));
  return p;
}

__device__ inline double i0_asym(double u) { return i0_asym_k<24>(u); }

// Series length for every u <= umax: the first dropped term c_K u^K is below
// 1e-17 for K = 10, 13, 16 up to u = 0.01, 0.02, 0.03 (x >= 100, 50, 33);
// otherwise the full 24 terms (below 1e-16 at u = 0.05, x = 20).
__device__ inline int asym_tier(double umax) {
  return umax <= 0.01 ? 0 : (umax <= 0.02 ? 1 : (umax <= 0.03 ? 2 : 3));
}

__device__ inline double i0_asym_tier(int tier, double u) {
  switch (tier) {
    case 0: return i0_asym_k<10>(u);
    case 1: return i0_asym_k<13>(u);
    case 2: return i0_asym_k<16>(u);
    default: return i0_asym_k<24>(u);
  }
}

// Series length for every y <= ymax: the first dropped term y^K / (K!)^2 is
// below 1e-17 (and I0 >= 1) for K = 8, 12, 16, 24 up to y = 0.106, 1.07, 4.00,
// 18.8; otherwise the full 40 terms (enough for y <= 100, i.e. x < 20).
__device__ inline int i0_tier(double ymax) {
  return ymax <= 0.106 ? 0 : (ymax <= 1.07 ? 1 : (ymax <= 4.0 ? 2 : (ymax <= 18.8 ? 3 : 4)));
}

__device__ inline double i0_series_tier(int tier, double y) {
  switch (tier) {
    case 0: return i0_series<8>(y);
    case 1: return i0_series<12>(y);
    case 2: return i0_series<16>(y);
    case 3: return i0_series<24>(y);
    default: return i0_series<40>(y);
  }
}

// Wave-uniform series tier for arguments up to x = z1 * r1max (z1 may differ
// between lanes): the largest need over the wave.
__device__ inline int wave_i0_tier(double z1, const LogI0Consts& C) {
  if (!(C.r1max > 0.0)) return 4;
  const double x = z1 * C.r1max;
  double y = 0.25 * x * x;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) y = fmax(y, __shfl_xor(y, o, 64));
  return __builtin_amdgcn_readfirstlane(i0_tier(y));
}

// Wave-uniform tier of the large-argument series for u = d / z1 up to
// dmax / z1 (only arguments x >= 20, u <= 0.05, take that series).
__device__ inline int wave_asym_tier(double z1, const LogI0Consts& C) {
  if (!(C.dmax > 0.0)) return 3;
  double u = z1 > 0.0 ? C.dmax / z1 : 1.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) u = fmax(u, __shfl_xor(u, o, 64));
  return __builtin_amdgcn_readfirstlane(asym_tier(u));
}

// ln I0(x) given x and u = 1/x (u is only used when x >= 20).
__device__ inline double log_i0_xu(double x, double u) {
  double arg, base, scale;
  if (x < 20.0) {
    const double y = 0.25 * x * x;
    arg = i0_series<40>(y);
    base = 0.0;
    scale = 1.0;
  } else {
    const double p = i0_asym(u);
    // x - ln(2 pi x)/2 + ln p = x + ln(p^2 u / (2 pi)) / 2
    arg = p * p * u * kInvTwoPi;
    base = x;
    scale = 0.5;
  }
  return fma(scale, log(arg), base);
}

__device__ inline double log_i0(double x) {
  return log_i0_xu(x, x >= 20.0 ? 1.0 / x : 0.0);
}

// Distance marginal over a grid, evaluated by one wave for one proposal:
//   LSE_j [ ln w_j - hh1 / (2 d_j^2) + ln I0(|Z1| / d_j) ],
// with the grid as records (d_j, 1/d_j, 1/(2 d_j^2), ln w_j).  Since
// ln I0(x) <= x, b_j = a_j + x_j with a_j = ln w_j - hh1 / (2 d_j^2) and
// x_j = |Z1| / d_j bounds term j from above, so every term is summed as
// exp(t_j - B) with B = max_j b_j and never overflows; the largest term is at
// least B - (x - ln I0(x)) at the maximising point, a gap below 15 for any
// finite x, so points with b_j < B - 60 (together below 1000 e^-45 of the sum)
// are skipped.  The 64 per-lane sums are merged by a fixed shuffle tree, so
// every lane returns the same, reproducible value.

// Wave-wide maximum of the bounds b_j.
__device__ inline double wave_dist_bound(double z1, double hh1, const double* __restrict__ tab, int n_dist, int lane) {
  double bmax = -INFINITY;
  for (int j = lane; j < n_dist; j += 64) {
    const double* r = tab + 4 * j;
    bmax = fmax(bmax, fma(-hh1, r[2], r[3]) + z1 * r[1]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) bmax = fmax(bmax, __shfl_xor(bmax, o, 64));
  return bmax;
}

__device__ inline double wave_sum(double s) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  return s;
}

// FP32 term of the single-precision form below: I0 from the FP32 fits,
// exp from the hardware 2^x; a = ln w - hh1 r2, x = |Z1| r1, B the bound.
__device__ inline float dist_term_f32(double a, double x, double bmax) {
  const float xf = (float)x;
  float p;
  double e;
  if (xf <= 8.0f) {
    const float sv = xf * xf * 0.015625f;
    p = kI0Small[kI0SmallDeg];
#pragma unroll
    for (int k = kI0SmallDeg - 1; k >= 0; --k) p = fmaf(p, sv, kI0Small[k]);
    e = a - bmax;
  } else {
    const float t = 8.0f * __builtin_amdgcn_rcpf(xf);
    float q = kI0Large[kI0LargeDeg];
#pragma unroll
    for (int k = kI0LargeDeg - 1; k >= 0; --k) q = fmaf(q, t, kI0Large[k]);
    p = q * __builtin_amdgcn_rsqf(xf);
    e = (a + x) - bmax;
  }
  return __builtin_amdgcn_exp2f((float)(e * kLog2E)) * p;
}

// FP64 form: I0 by its power series in y = x^2/4 below x = 20 (40 terms) and
// by the asymptotic series e^x / sqrt(2 pi x) sum_k c_k x^-k above (24 terms).
// A term whose bound a + x lies more than 35 below B is at most e^-20 of the
// sum (ln I0(x) >= x - 15 at the bound's maximiser, so the sum is at least
// e^(B - 15)); such terms take the FP32 form (relative error below 4e-6, most
// of it from the exponent rounded to FP32), which moves the sum by less than
// n_dist e^-20 4e-6 of itself (1e-11 at 1000 grid points).  Lanes walk
// consecutive grid points, so a wave mostly takes one form at a time.
__device__ inline double wave_dist_lse(double z1, double hh1, const double* __restrict__ tab, int n_dist, int lane,
                                       const LogI0Consts& C) {
  const double bmax = wave_dist_bound(z1, hh1, tab, n_dist, lane);
  const double cut = bmax - 60.0, fine = bmax - 35.0;
  const double iz = z1 > 0.0 ? 1.0 / z1 : 0.0;
  const int tier = wave_i0_tier(z1, C), atier = wave_asym_tier(z1, C);
  double s = 0.0;
  for (int j = lane; j < n_dist; j += 64) {
    const double* r = tab + 4 * j;
    const double a = fma(-hh1, r[2], r[3]);
    const double x = z1 * r[1];
    if (a + x < cut) continue;
    if (a + x < fine) {
      s += (double)dist_term_f32(a, x, bmax);
      continue;
    }
    double v, e;
    if (x < 20.0) {
      v = i0_series_tier(tier, 0.25 * x * x);
      e = a - bmax;
    } else {
      const double u = r[0] * iz;  // 1 / x
      const double p = i0_asym_tier(atier, u);
      v = p * sqrt(u * kInvTwoPi);
      e = (a + x) - bmax;
    }
    s = fma(exp_nonpos(e, C.exp2_64), v, s);
  }
  return bmax + log(wave_sum(s));
}

// Single-precision form (the mixed path): the exponent arguments a_j, x_j and
// t_j - B stay FP64; I0 comes from the FP32 polynomial fits of gw_i0_fit.h
// (relative error below 4e-7 after FP32 rounding) and exp from the hardware
// 2^x, the per-lane sums are FP32 and the tree FP64.
__device__ inline double wave_dist_lse_f32(double z1, double hh1, const double* __restrict__ tab, int n_dist,
                                           int lane) {
  const double bmax = wave_dist_bound(z1, hh1, tab, n_dist, lane);
  const double cut = bmax - 60.0;
  float s = 0.0f;
  for (int j = lane; j < n_dist; j += 64) {
    const double* r = tab + 4 * j;
    const double a = fma(-hh1, r[2], r[3]);
    const double x = z1 * r[1];
    if (a + x < cut) continue;
    const float xf = (float)x;
    float p;
    double e;
    if (xf <= 8.0f) {
      const float sv = xf * xf * 0.015625f;
      p = kI0Small[kI0SmallDeg];
#pragma unroll
      for (int k = kI0SmallDeg - 1; k >= 0; --k) p = fmaf(p, sv, kI0Small[k]);
      e = a - bmax;
    } else {
      const float t = 8.0f * __builtin_amdgcn_rcpf(xf);
      float q = kI0Large[kI0LargeDeg];
#pragma unroll
      for (int k = kI0LargeDeg - 1; k >= 0; --k) q = fmaf(q, t, kI0Large[k]);
      p = q * __builtin_amdgcn_rsqf(xf);
      e = (a + x) - bmax;
    }
    s = fmaf(__builtin_amdgcn_exp2f((float)(e * kLog2E)), p, s);
  }
  return bmax + log(wave_sum((double)s));
}

// Sliced forms of the distance marginal: one proposal per lane, and the
// waves of a workgroup share the same 64 proposals, each wave taking a slice
// [j0, j1) of the grid.  All lanes of a wave walk their slice together, so
// each grid record is a wave-uniform (scalar) load shared by 64 proposals
// instead of a separate vector load per lane.  The caller combines the slice
// maxima (order-independent) and then the slice sums in a fixed order; the
// bound, cut and term arithmetic are those of the wave forms above.
__device__ inline double slice_dist_bound(double z1, double hh1, const double* __restrict__ tab, int j0, int j1) {
  double bmax = -INFINITY;
  for (int j = j0; j < j1; ++j) {
    const double* r = tab + 4 * j;
    bmax = fmax(bmax, fma(-hh1, r[2], r[3]) + z1 * r[1]);
  }
  return bmax;
}

// sum_j exp(t_j - bmax) over the slice (FP64 form; terms more than 35
// below the bound in FP32, as in wave_dist_lse).
__device__ inline double slice_dist_sum(double z1, double hh1, double bmax, const double* __restrict__ tab, int j0,
                                        int j1, const LogI0Consts& C) {
  const double cut = bmax - 60.0, fine = bmax - 35.0;
  const double iz = z1 > 0.0 ? 1.0 / z1 : 0.0;
  const int tier = wave_i0_tier(z1, C), atier = wave_asym_tier(z1, C);
  double s = 0.0;
  for (int j = j0; j < j1; ++j) {
    const double* r = tab + 4 * j;
    const double a = fma(-hh1, r[2], r[3]);
    const double x = z1 * r[1];
    if (a + x < cut) continue;
    if (a + x < fine) {
      s += (double)dist_term_f32(a, x, bmax);
      continue;
    }
    double v, e;
    if (x < 20.0) {
      v = i0_series_tier(tier, 0.25 * x * x);
      e = a - bmax;
    } else {
      const double u = r[0] * iz;  // 1 / x
      const double p = i0_asym_tier(atier, u);
      v = p * sqrt(u * kInvTwoPi);
      e = (a + x) - bmax;
    }
    s = fma(exp_nonpos(e, C.exp2_64), v, s);
  }
  return s;
}

// Same sum, single-precision form.
__device__ inline double slice_dist_sum_f32(double z1, double hh1, double bmax, const double* __restrict__ tab,
                                            int j0, int j1) {
  const double cut = bmax - 60.0;
  float s = 0.0f;
  for (int j = j0; j < j1; ++j) {
    const double* r = tab + 4 * j;
    const double a = fma(-hh1, r[2], r[3]);
    const double x = z1 * r[1];
    if (a + x < cut) continue;
    const float xf = (float)x;
    float p;
    double e;
    if (xf <= 8.0f) {
      const float sv = xf * xf * 0.015625f;
      p = kI0Small[kI0SmallDeg];
#pragma unroll
      for (int k = kI0SmallDeg - 1; k >= 0; --k) p = fmaf(p, sv, kI0Small[k]);
      e = a - bmax;
    } else {
      const float t = 8.0f * __builtin_amdgcn_rcpf(xf);
      float q = kI0Large[kI0LargeDeg];
#pragma unroll
      for (int k = kI0LargeDeg - 1; k >= 0; --k) q = fmaf(q, t, kI0Large[k]);
      p = q * __builtin_amdgcn_rsqf(xf);
      e = (a + x) - bmax;
    }
    s = fmaf(__builtin_amdgcn_exp2f((float)(e * kLog2E)), p, s);
  }
  return (double)s;
}

// Workgroup-level driver: waves w = 0 .. nw-1 of the block share 64
// proposals (lane = proposal); red is LDS scratch of nw x 64 doubles.
// Returns the log-sum-exp in every lane of wave 0 (other waves return 0).
template <int PREC>
__device__ inline double block_dist_lse(double z1, double hh1, const double* __restrict__ tab, int n_dist, int nw,
                                        double* red, const LogI0Consts& C) {
  const int lane = threadIdx.x & 63;
  // wave index, made visibly wave-uniform so that the grid loads are scalar
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int per = (n_dist + nw - 1) / nw;
  const int j0 = w * per < n_dist ? w * per : n_dist;
  const int j1 = j0 + per < n_dist ? j0 + per : n_dist;
  red[w * 64 + lane] = slice_dist_bound(z1, hh1, tab, j0, j1);
  __syncthreads();
  double bmax = -INFINITY;
  for (int v = 0; v < nw; ++v) bmax = fmax(bmax, red[v * 64 + lane]);
  __syncthreads();
  red[w * 64 + lane] = PREC == 0 ? slice_dist_sum(z1, hh1, bmax, tab, j0, j1, C)
                                 : slice_dist_sum_f32(z1, hh1, bmax, tab, j0, j1);
  __syncthreads();
  double s = 0.0;
  if (w == 0)
    for (int v = 0; v < nw; ++v) s += red[v * 64 + lane];
  __syncthreads();
  return w == 0 ? bmax + log(s) : 0.0;
}

}  // namespace gw
