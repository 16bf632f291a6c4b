// Index maps and register passes of the time-grid transform (gw_tgrid.hip),
// host and device: L = D1 D2 16 points, an in-place decimation-in-frequency
// FFT in three passes.
//   pass 1, lane r < L / D1: DFT over x[r + (L / D1) q], q < D1, output k1
//           times exp(-2 pi i r k1 / L), stored at r + (L / D1) k1;
//   pass 2, lane n3 + 16 k1 (n3 < 16, k1 < D1): DFT over the D2 values at
//           n3 + 16 q + (L / D1) k1, output k2 times exp(-2 pi i n3 k2 / (16 D2)),
//           stored in place;
//   pass 3, lane g < L / 16: DFT over the 16 values at 16 g + n3; output k3 is
//           X[tg_owned(L, D1, D2, g, k3)].
#pragma once

#include <math.h>

#include <vector>

#include "gw_fft.h"

namespace gw {

constexpr int kTgMaxL = 4096;

// LDS position of element i: one pad element per 16.
__host__ __device__ inline int tg_pad(int i) { return i + (i >> 4); }

// The transform index that lane `lane` (< L / 16) holds in output slot k3 of
// the last pass: k1 + D1 k2 + (L / 16) k3 with k1 = lane / D2, k2 = lane mod D2.
__host__ __device__ inline int tg_owned(int L, int D1, int D2, int lane, int k3) {
  return lane / D2 + D1 * (lane % D2) + (L / 16) * k3;
}

// Pass radices for a length L = 2^q, 16 <= L <= 4096.
inline bool tgrid_plan(int L, int* D1, int* D2) {
  if (L < 16 || L > kTgMaxL || (L & (L - 1)) != 0) return false;
  if (L >= 256) {
    *D1 = L / 256;
    *D2 = 16;
  } else {
    *D1 = 1;
    *D2 = L / 16;
  }
  return true;
}

// First pass on one lane's D1 inputs (only v[0 .. NZ) may be nonzero, the
// rest hold zero), w = exp(-2 pi i r / L); outputs in natural order.
template <int D1, int NZ>
__host__ __device__ inline void tg_pass1(double2* v, double2 w) {
  if constexpr (D1 > 1) {
    if constexpr (D1 == 16) {
      Dft<16>::template run_slots_nz<NZ>(v);
    } else {
      Dft<D1>::run_slots(v);
    }
    double2 o[D1];
#pragma unroll
    for (int k = 0; k < D1; ++k) o[k] = v[dft_slot<D1>(k)];
    double2 t = w;
#pragma unroll
    for (int k = 1; k < D1; ++k) {
      o[k] = c_mul(o[k], t);
      if (k + 1 < D1) t = c_mul(t, w);
    }
#pragma unroll
    for (int k = 0; k < D1; ++k) v[k] = o[k];
  }
}

// Second pass on one lane's D2 values, w = exp(-2 pi i n3 / (16 D2)).
template <int D2>
__host__ __device__ inline void tg_pass2(double2* v, double2 w) {
  if constexpr (D2 > 1) {
    Dft<D2>::run_slots(v);
    double2 o[D2];
#pragma unroll
    for (int k = 0; k < D2; ++k) o[k] = v[dft_slot<D2>(k)];
    double2 t = w;
#pragma unroll
    for (int k = 1; k < D2; ++k) {
      o[k] = c_mul(o[k], t);
      if (k + 1 < D2) t = c_mul(t, w);
    }
#pragma unroll
    for (int k = 0; k < D2; ++k) v[k] = o[k];
  }
}

// J_n(x) by its power series (|x| <= pi / 2 here: the terms fall by at least
// (x / 2)^2 / k at step k, so the sum settles in a dozen terms).
inline double tgrid_bessel_jn(int n, double x) {
  const long double h = 0.5L * (long double)x;
  long double t = 1.0L;
  for (int i = 1; i <= n; ++i) t *= h / (long double)i;
  long double s = t;
  for (int k = 1; k < 60; ++k) {
    t *= -(h * h) / ((long double)k * (long double)(n + k));
    s += t;
    if (fabsl(t) <= 1e-22L * fabsl(s)) break;
  }
  return (double)s;
}

// Expansion orders for a grid of |j| <= jmax on a length-L transform: 12 when
// the dropped orders' bound 2 (phi / 2)^12 / 12! at phi = pi jmax / L is at
// most 2e-11, else 16.
inline int tgrid_orders(int L, int jmax) {
  const double phi = 3.141592653589793 * (double)jmax / (double)L;
  double b = 2.0;
  for (int i = 1; i <= 12; ++i) b *= 0.5 * phi / (double)i;
  return b <= 2e-11 ? 12 : 16;
}

// Coefficient table [K][256][16]: eps_m J_m(pi j / L) with the sign of (-i)^m
// folded in (+ for m mod 4 in {0, 1}, - otherwise), for lane l's output slot
// k3 at (m 256 + l) 16 + k3; zero where the slot's |j| exceeds jmax.
inline void tgrid_coefficients(int L, int jmax, int K, std::vector<double>* out) {
  int D1 = 1, D2 = 1;
  out->assign((size_t)K * 16 * 256, 0.0);
  if (!tgrid_plan(L, &D1, &D2)) return;
  for (int lane = 0; lane < L / 16; ++lane)
    for (int k3 = 0; k3 < 16; ++k3) {
      const int X = tg_owned(L, D1, D2, lane, k3);
      const int j = X <= jmax ? X : X - L;
      if (j < -jmax || j > jmax) continue;
      const double phi = 3.141592653589793 * (double)j / (double)L;
      for (int m = 0; m < K; ++m) {
        const double sgn = (m & 3) < 2 ? 1.0 : -1.0;
        (*out)[((size_t)m * 256 + lane) * 16 + k3] = sgn * (m == 0 ? 1.0 : 2.0) * tgrid_bessel_jn(m, phi);
      }
    }
}

// Chebyshev values T_m(s), m < K (T_0 = 1, T_1 = s, T_{m+1} = 2 s T_m - T_{m-1}).
inline void tgrid_basis_at(double s, int K, double* t) {
  double a = 1.0, b = s;
  for (int m = 0; m < K; ++m) {
    t[m] = a;
    const double c = 2.0 * s * b - a;
    a = b;
    b = c;
  }
}

// The same at s = (j - (blk - 1) / 2) / (blk / 2) for j < blk: [blk][K].
inline void tgrid_basis(int blk, int K, std::vector<double>* out) {
  out->assign((size_t)blk * K, 0.0);
  const double cen = 0.5 * (blk - 1), hinv = 2.0 / blk;
  for (int j = 0; j < blk; ++j) tgrid_basis_at(((double)j - cen) * hinv, K, out->data() + (size_t)j * K);
}

}  // namespace gw
