// Small in-register DFTs and one Stockham autosort pass, FP64 complex.
//
// dft<R>(v) replaces v[0..R) by X_k = sum_n v_n exp(-2 pi i n k / R) (natural
// order in and out), R in {2, 4, 8, 16}, by radix-2 decimation in time over
// a radix-4 base.  A Stockham pass of radix R over L points with span ns
// (the product of the earlier passes' radices) takes butterfly j < L / R from
// x[j + q L / R], q < R, multiplies input q by exp(-2 pi i (j mod ns) q /
// (ns R)), transforms, and writes output q to y[(j - j mod ns) R + j mod ns +
// q ns]; passes of radices R1 R2 ... = L in that order give the DFT of
// length L in natural order.
#pragma once

#include <hip/hip_runtime.h>

namespace gw {

__host__ __device__ inline double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 c_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a times -i
__host__ __device__ inline double2 c_mul_mi(double2 a) { return make_double2(a.y, -a.x); }

template <int R>
struct Dft;

template <>
struct Dft<2> {
  __host__ __device__ static inline void run(double2* v) {
    const double2 a = v[0], b = v[1];
    v[0] = c_add(a, b);
    v[1] = c_sub(a, b);
  }
  __host__ __device__ static inline void run_slots(double2* v) { run(v); }
};

template <>
struct Dft<4> {
  __host__ __device__ static inline void run(double2* v) {
    const double2 a0 = c_add(v[0], v[2]), a1 = c_sub(v[0], v[2]);
    const double2 a2 = c_add(v[1], v[3]), a3 = c_mul_mi(c_sub(v[1], v[3]));
    v[0] = c_add(a0, a2);
    v[1] = c_add(a1, a3);
    v[2] = c_sub(a0, a2);
    v[3] = c_sub(a1, a3);
  }
  __host__ __device__ static inline void run_slots(double2* v) { run(v); }
};

// exp(-2 pi i k / 16), k = 0 .. 15
__host__ __device__ inline double2 w16(int k) {
  constexpr double c1 = 0.92387953251128674, s1 = 0.38268343236508977, h = 0.70710678118654752;
  switch (k) {
    case 0: return make_double2(1.0, 0.0);
    case 1: return make_double2(c1, -s1);
    case 2: return make_double2(h, -h);
    case 3: return make_double2(s1, -c1);
    case 4: return make_double2(0.0, -1.0);
    case 5: return make_double2(-s1, -c1);
    case 6: return make_double2(-h, -h);
    case 7: return make_double2(-c1, -s1);
    case 8: return make_double2(-1.0, 0.0);
    case 9: return make_double2(-c1, s1);
    default: {  // k = 10 .. 15: conj(w16(16 - k))
      const double2 w = w16(16 - k);
      return make_double2(w.x, -w.y);
    }
  }
}

// DFT4 of t[0..4) with only the leading NZ inputs nonzero (NZ in {1, 2, 4}).
template <int NZ>
__host__ __device__ inline void dft4_nz(double2* t) {
  if constexpr (NZ == 1) {
    t[1] = t[0];
    t[2] = t[0];
    t[3] = t[0];
  } else if constexpr (NZ == 2) {
    const double2 a = t[0], b = t[1], mb = c_mul_mi(b);
    t[0] = c_add(a, b);
    t[1] = c_add(a, mb);
    t[2] = c_sub(a, b);
    t[3] = c_sub(a, mb);
  } else {
    Dft<4>::run(t);
  }
}

// Radix 8 and 16 in place as (R / 4) x 4: with n = n1 + (R / 4) n2 and
// k = 4 k1 + k2, DFT4 over n2 for each n1, twiddle by exp(-2 pi i n1 k2 / R),
// then DFT over n1 for each k2.  Output k lands in slot slot<R>(k) of v.
template <int R>
__host__ __device__ constexpr int dft_slot(int k) {
  return R == 16 ? 4 * (k & 3) + (k >> 2) : (R == 8 ? 2 * (k & 3) + (k >> 2) : k);
}

template <int R>
struct Dft {
  // in-place transform leaving output k in v[dft_slot<R>(k)]
  __host__ __device__ static inline void run_slots(double2* v) {
    constexpr int A = R / 4;  // n1 range
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) {
      double2 t[4] = {v[n1], v[n1 + A], v[n1 + 2 * A], v[n1 + 3 * A]};
      Dft<4>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[n1 + A * k2] = (n1 * k2) ? c_mul(w16((16 / R) * n1 * k2), t[k2]) : t[k2];
    }
    // slot n1 + A k2 now holds y[n1][k2]; transform over n1 for each k2
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      double2 t[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) t[n1] = v[n1 + A * k2];
      Dft<A>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) v[A * k2 + k1] = t[k1];  // X[4 k1 + k2]
    }
  }
  // run_slots for inputs of which only v[0 .. NZ) may be nonzero (R = 16,
  // NZ in {1, 2, 4, 8, 16}; the others must hold zero): the work on the known
  // zeros is skipped
  template <int NZ>
  __host__ __device__ static inline void run_slots_nz(double2* v) {
    static_assert(R == 16, "pruned form for radix 16 only");
    constexpr int N1 = NZ < 4 ? NZ : 4;        // rows n1 holding a nonzero input
    constexpr int N2 = NZ <= 4 ? 1 : NZ / 4;   // nonzero inputs per such row
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      double2 t[4] = {v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]};
      dft4_nz<N2>(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[n1 + 4 * k2] = (n1 * k2) ? c_mul(w16(n1 * k2), t[k2]) : t[k2];
    }
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      double2 t[4] = {v[4 * k2], v[4 * k2 + 1], v[4 * k2 + 2], v[4 * k2 + 3]};
      dft4_nz<N1>(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) v[4 * k2 + k1] = t[k1];
    }
  }
  // natural order
  __host__ __device__ static inline void run(double2* v) {
    run_slots(v);
    double2 o[R];
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = v[dft_slot<R>(k)];
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = o[k];
  }
};

}  // namespace gw
