// Grid sum over coalescence-time shifts from block moments (Sec. III.A and the
// appendix on grid marginalisations), shared by the full-band and heterodyned
// time marginals.
//
// The shifts are t_j = j delta / R, |j| <= jmax = J R, with delta the
// segment's sampling interval 1 / (N df).  A frequency on the fine grid,
// f = f_k0 + k df, is split as k = b B + (B - 1) / 2 + s B / 2 with B = N / P
// bins per block (P a power of two >= 2 J + 1) and s in [-1, 1], so that
//   exp(-2 pi i f t_j) = exp(-2 pi i f_0 t_j) exp(-2 pi i b j / L) exp(-i phi_j s),
// L = P R, phi_j = pi j / L, |phi_j| < pi / 2, f_0 the first block's centre.
// The last factor is expanded in Chebyshev polynomials of s (the Jacobi-Anger
// expansion), exp(-i phi s) = sum_n eps_n (-i)^n J_n(phi) T_n(s), eps_0 = 1 and
// eps_n = 2 otherwise; with M_bn = sum_{k in block b} T_n(s_k) y_k (y the
// per-bin overlap weights of the full band, or the per-edge weights of the
// heterodyned bins),
//   Z(t_j) = exp(-2 pi i f_0 t_j) sum_{n < K} eps_n (-i)^n J_n(phi_j) F_n(j),
//   F_n(j) = sum_b M_bn exp(-2 pi i b j / L),
// one length-L DFT per order.  |T_n| <= 1 and |J_n(phi)| <= (phi / 2)^n / n!,
// so the dropped orders stay below 2 (phi / 2)^K / K! of the sum of |y|; the
// host takes K = 12 when that is below 2e-11 (|phi| up to 1.27, every grid of
// the default window) and K = 16 otherwise (below 3e-15 at pi / 2).  The
// leading factor has unit modulus.
//
// k_tgrid: one workgroup (256 lanes) per row.  Per order, an in-place
// decimation-in-frequency FFT of L = D1 D2 16 points (D1 = L / 256 for
// L >= 256, else D1 = 1 and D2 = L / 16) in three passes: the first reads the
// moments straight from memory (blocks at or beyond n_blk are zero; for
// L = 4096 the radix-16 butterfly skips the inputs known to be zero), the
// second works in LDS, and the third leaves each lane its 16 outputs in
// registers, where they are weighted by the expansion coefficients (a table
// per grid) and accumulated.  The LDS buffer stores element i at
// i + floor(i / 16), which keeps all three access patterns free of bank
// conflicts.  Twiddles are powers of one root of unity per lane, formed by
// repeated products.  Then ln I0(|Z|) - <h|h>(t_j) / 2 and a fixed-order
// log-sum-exp.  For the heterodyned bins the norm also depends on t_j:
// <h|h>(t_j) = hhc + Re exp(-2 pi i c u_j) sum_{m < MH} (-i x_j)^m / m! S_m,
// u_j = j / (N R) (fine-grid cycles), x_j = 2 pi hw u_j, with the bin widths
// dk_e = c + hw sigma_e expanded about their centre c and S_m the per-row
// moments sum_e sigma_e^m V_e (partial sums over edge chunks, added here in
// chunk order).
#include <math.h>

#include <algorithm>
#include <vector>

#include "gw_ctx.h"
#include "gw_fft.h"
#include "gw_tgrid.h"

namespace gw {

constexpr int kTgBuf = kTgMaxL + kTgMaxL / 16;  // padded LDS buffer

// w2 = exp(-2 pi i n3 / (16 D2)) for the lane's n3 = tid mod 16
template <int D2>
__device__ inline void tg_lds_pass2(double2* __restrict__ buf, int tid, int D1, int S1, double2 w2) {
  if (tid < 16 * D1) {
    const int n3 = tid & 15, k1 = tid >> 4;
    // element n3 + 16 q + S1 k1 sits at tg_pad(n3 + S1 k1) + 17 q (S1 is a
    // multiple of 16)
    const int pb = tg_pad(n3 + S1 * k1);
    double2 v[D2];
#pragma unroll
    for (int q = 0; q < D2; ++q) v[q] = buf[pb + 17 * q];
    tg_pass2<D2>(v, w2);
#pragma unroll
    for (int q = 0; q < D2; ++q) buf[pb + 17 * q] = v[q];
  }
}

constexpr int kTgXcds = 8;  // XCDs of the GPU (workgroups are dealt to them in turn)

struct TgKernelArgs {
  const double2* mom;  // element (p, m, b) at p mom_rs + (m n_blk + b) mom_es
  int64_t mom_rs, mom_es;
  int64_t n;
  int n_blk, L, D2, K, jmax;
  const double* ccoef;  // [K][256][16]
  const double* coef;
  int64_t ld;
  double dd;
  double* logl;
  const double* hhc;
  const double2* hpart;
  int n_hch, mh;
  double hw_step;
  int64_t c2, cden;
  double* zout;
  double f0_num, f0_den;
  int S;            // order groups per row (1: one workgroup per row finishes it)
  double2* zpart;   // S > 1: [S][n][2 jmax + 1] the groups' partial Z(t_j)
};

// Epilogue of one row: Z(t_j) in buf [0, nt) in grid order (written before
// the call, made visible by its first barrier); <h|h>(t_j), the staged
// values (zout), ln I0(|Z|) - <h|h>/2 and a fixed-order log-sum-exp into
// logl[p].  All 256 threads of the workgroup call it.
template <int HET>
__device__ inline void tg_epilogue(const TgKernelArgs& a, int64_t p, const double2* __restrict__ buf,
                                   double2* __restrict__ sm, double* __restrict__ sinv, double* __restrict__ red,
                                   double* __restrict__ red2) {
  const int tid = threadIdx.x;
  const int nt = 2 * a.jmax + 1;
  const bool valid = a.coef[C_VALID * a.ld + p] != 0.0;
  double hh = 0.0;
  if (HET) {
    hh = a.hhc[p];
    // this row's H moments, summed over the edge chunks: thread (g, q)
    // adds chunks g, g + 4, ... of moment q, and the four sums are added in
    // order g = 0 .. 3 (red and red2 hold them; mh <= kTgHMax <= 64)
    {
      const int q = tid & 63, g = tid >> 6;
      double2 s = make_double2(0.0, 0.0);
      if (q < a.mh)
        for (int c = g; c < a.n_hch; c += 4) s = c_add(s, a.hpart[((int64_t)c * a.n + p) * a.mh + q]);
      red[tid] = s.x;
      red2[tid] = s.y;
      __syncthreads();
      if (tid < a.mh) {
        sm[tid] = make_double2(((red[tid] + red[tid + 64]) + red[tid + 128]) + red[tid + 192],
                               ((red2[tid] + red2[tid + 64]) + red2[tid + 128]) + red2[tid + 192]);
        sinv[tid] = 1.0 / (double)(tid + 1);
      }
    }
  } else {
    hh = a.coef[C_HH * a.ld + p];
  }
  // exp(-2 pi i c u_j) at this lane's first point, and its step over 256
  // points (a rotation applied once per point below)
  double cs = 1.0, sn = 0.0, rc = 1.0, rs = 0.0;
  if (HET) {
    const int64_t num = (a.c2 * (int64_t)(tid - a.jmax)) % a.cden;
    sincospi(-2.0 * (double)num / (double)a.cden, &sn, &cs);
    const int64_t stp = (a.c2 * 256) % a.cden;
    sincospi(-2.0 * (double)stp / (double)a.cden, &rs, &rc);
  }
  __syncthreads();
  double run_mx = -INFINITY, run_acc = 0.0;
  for (int jj = tid; jj < nt; jj += 256) {
    const int j = jj - a.jmax;
    const double2 z = buf[jj];
    double hj = hh;
    if (HET) {
      const double xq = a.hw_step * (double)j;
      double tr = 0.0, ti = 0.0;
      for (int q = a.mh - 1; q >= 0; --q) {
        const double qq = xq * sinv[q];
        const double nr = fma(qq, ti, sm[q].x), ni = fma(-qq, tr, sm[q].y);
        tr = nr;
        ti = ni;
      }
      hj += cs * tr - sn * ti;
      const double c2_ = cs * rc - sn * rs;
      sn = cs * rs + sn * rc;
      cs = c2_;
    }
    if (a.zout) {
      const double cyc = (double)j * a.f0_num / a.f0_den;
      double sn, cs;
      sincospi(2.0 * (cyc - rint(cyc)), &sn, &cs);
      double* zo = a.zout + (p * nt + jj) * 3;
      zo[0] = valid ? cs * z.x + sn * z.y : NAN;
      zo[1] = cs * z.y - sn * z.x;
      zo[2] = hj;
    }
    const double v = -0.5 * hj + log_i0(sqrt(z.x * z.x + z.y * z.y));
    if (v > run_mx) {
      run_acc = run_acc * exp(run_mx - v) + 1.0;
      run_mx = v;
    } else if (!(v == -INFINITY)) {
      run_acc += exp(v - run_mx);
    }
  }
  // merge the lanes' (maximum, scaled sum) pairs in a fixed order
  red[tid] = run_mx;
  red2[tid] = run_acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      const double ma = red[tid], mb = red[tid + s];
      const double mm = fmax(ma, mb);
      if (mm > -INFINITY) {
        red2[tid] = red2[tid] * exp(ma - mm) + red2[tid + s] * exp(mb - mm);
        red[tid] = mm;
      }
    }
    __syncthreads();
  }
  if (tid == 0) a.logl[p] = valid ? -0.5 * a.dd + red[0] + log(red2[0]) - log((double)nt) : -INFINITY;
}

// mom: complex moments, row p, order m, block b at p mom_rs + (m n_blk + b)
// mom_es (row-major [n][K][n_blk]: (K n_blk, 1); row fastest [K][n_blk][n]:
// (1, n)).
// ccoef: eps_m J_m(phi_j) for lane l's output slot k3 at (m 256 + l) 16 + k3,
// with the sign of (-i)^m folded in (+ for m mod 4 in {0, 1}, - otherwise)
// and zero where |j| > jmax.  HET = 0: <h|h> = coef[C_HH]; HET = 1:
// <h|h>(t_j) as above from hhc [n], the H moments hpart [n_hch][n][mh]
// complex, hw_step = 2 pi hw / (N R), c2 = 2 c and cden = 2 N R
// (exp(-2 pi i c u_j) = exp(-2 pi i (c2 j mod cden) / cden)).  zout (else
// NULL): [n][2 jmax + 1][3] = (Re Z(t_j), Im Z(t_j), <h|h>(t_j)), Re NaN for
// unphysical rows, with f_0 t_j = j f0_num / f0_den cycles.
template <int HET, int D1, int NZ>
__global__ void __launch_bounds__(256, 2) k_tgrid(TgKernelArgs a) {
  __shared__ double2 buf[kTgBuf];
  __shared__ double2 sm[kTgHMax];
  __shared__ double sinv[kTgHMax];  // 1 / (q + 1)
  __shared__ double red[256], red2[256];
  // Workgroups are dealt to the 8 XCDs in turn, each with its own L2; in the
  // rows-fastest moment layout neighbouring rows share cache lines, so there
  // workgroup i takes row (i mod 8) span + i / 8 and the rows of one XCD are
  // consecutive (row-major moments: row i).
  // With S > 1 order groups, workgroup i takes group i mod S of row slot
  // i / S (the groups' partial sums are added by k_tgrid_fin).
  const int g = (int)(blockIdx.x % (unsigned)a.S);
  const int64_t w = blockIdx.x / (unsigned)a.S;
  const int64_t span = (a.n + kTgXcds - 1) / kTgXcds;
  const int64_t p = a.mom_es != 1 ? (w % kTgXcds) * span + w / kTgXcds : w;
  if (p >= a.n) return;  // whole workgroup, before any barrier
  const int tid = threadIdx.x;
  const int L = a.L, D2 = D1 > 1 ? 16 : a.D2, K = a.K;
  const int S1 = L / D1;  // = 16 D2
  const int nt = 2 * a.jmax + 1;
  const double2* __restrict__ mrow = a.mom + p * a.mom_rs;
  const int64_t es = a.mom_es;
  const bool on1 = tid < S1, on3 = tid < L / 16;
  double2 w1 = make_double2(1.0, 0.0), w2;
  if (D1 > 1) {
    double s, c;
    sincospi(-2.0 * (double)tid / (double)L, &s, &c);
    w1 = make_double2(c, s);
  }
  {
    double s, c;
    sincospi(-2.0 * (double)(tid & 15) / (double)(16 * D2), &s, &c);
    w2 = make_double2(c, s);
  }
  double ar[16], ai[16];
#pragma unroll
  for (int o = 0; o < 16; ++o) ar[o] = ai[o] = 0.0;
  // the first pass's inputs of the current order (prefetched one order
  // ahead when they are few)
  constexpr bool kPrefetch = NZ <= 4;
  double2 x[NZ];
  auto load = [&](int m) {
    const double2* __restrict__ src = mrow + (int64_t)m * a.n_blk * es;
#pragma unroll
    for (int q = 0; q < NZ; ++q) {
      const int b = tid + S1 * q;
      x[q] = (on1 && b < a.n_blk) ? src[b * es] : make_double2(0.0, 0.0);
    }
  };
  const int m_lo = g * (K / a.S), m_hi = m_lo + K / a.S;  // this group's orders
  if (kPrefetch) load(m_lo);
  for (int m = m_lo; m < m_hi; ++m) {
    // The twiddle powers are formed afresh in every order: an empty asm
    // statement marks the roots as changing here, so the compiler does not
    // hoist 30 loop-invariant powers out of the loop (they would spill).
    asm volatile("" : "+v"(w1.x), "+v"(w1.y), "+v"(w2.x), "+v"(w2.y));
    if (!kPrefetch) load(m);
    double2 v[D1];
#pragma unroll
    for (int q = 0; q < D1; ++q) v[q] = q < NZ ? x[q] : make_double2(0.0, 0.0);
    if (kPrefetch && m + 1 < m_hi) load(m + 1);
    tg_pass1<D1, NZ>(v, w1);
    __syncthreads();  // the previous order's last-pass reads are done
    if (on1) {
      const int pb = tg_pad(tid);
#pragma unroll
      for (int k = 0; k < D1; ++k) buf[pb + 17 * (S1 / 16) * k] = v[k];
    }
    __syncthreads();
    if constexpr (D1 > 1) {
      tg_lds_pass2<16>(buf, tid, D1, S1, w2);  // L >= 512: D2 = 16
    } else {
      switch (D2) {
        case 16: tg_lds_pass2<16>(buf, tid, D1, S1, w2); break;
        case 8: tg_lds_pass2<8>(buf, tid, D1, S1, w2); break;
        case 4: tg_lds_pass2<4>(buf, tid, D1, S1, w2); break;
        case 2: tg_lds_pass2<2>(buf, tid, D1, S1, w2); break;
        default: break;
      }
    }
    __syncthreads();
    if (on3) {
      double2 f[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) f[q] = buf[17 * tid + q];
      Dft<16>::run_slots(f);
      const double* __restrict__ cm = a.ccoef + ((int64_t)m * 256 + tid) * 16;
      if ((m & 1) == 0) {
#pragma unroll
        for (int k3 = 0; k3 < 16; ++k3) {
          const double t = cm[k3];
          const double2 z = f[dft_slot<16>(k3)];
          ar[k3] = fma(t, z.x, ar[k3]);
          ai[k3] = fma(t, z.y, ai[k3]);
        }
      } else {
#pragma unroll
        for (int k3 = 0; k3 < 16; ++k3) {
          const double t = cm[k3];
          const double2 z = f[dft_slot<16>(k3)];
          ar[k3] = fma(t, z.y, ar[k3]);
          ai[k3] = fma(-t, z.x, ai[k3]);
        }
      }
    }
  }
  if (a.S > 1) {  // this group's partial Z(t_j), finished by k_tgrid_fin
    if (on3) {
      double2* __restrict__ zp = a.zpart + ((int64_t)g * a.n + p) * nt + a.jmax;
#pragma unroll
      for (int k3 = 0; k3 < 16; ++k3) {
        const int X = tg_owned(L, D1, D2, tid, k3);
        const int j = X <= a.jmax ? X : X - L;
        if (j >= -a.jmax && j <= a.jmax) zp[j] = make_double2(ar[k3], ai[k3]);
      }
    }
    return;
  }
  // the finished Z(t_j) go to the buffer in grid order (nt <= L points), read
  // back by the epilogue in a plain loop
  __syncthreads();
  if (on3) {
#pragma unroll
    for (int k3 = 0; k3 < 16; ++k3) {
      const int X = tg_owned(L, D1, D2, tid, k3);
      const int j = X <= a.jmax ? X : X - L;
      if (j >= -a.jmax && j <= a.jmax) buf[j + a.jmax] = make_double2(ar[k3], ai[k3]);
    }
  }
  tg_epilogue<HET>(a, p, buf, sm, sinv, red, red2);
}

// k_tgrid_fin: one workgroup per row adds the S groups' partial Z(t_j) in
// group order and runs the epilogue.
template <int HET>
__global__ void __launch_bounds__(256) k_tgrid_fin(TgKernelArgs a) {
  __shared__ double2 buf[kTgMaxL];
  __shared__ double2 sm[kTgHMax];
  __shared__ double sinv[kTgHMax];
  __shared__ double red[256], red2[256];
  const int64_t p = blockIdx.x;
  const int nt = 2 * a.jmax + 1;
  for (int jj = threadIdx.x; jj < nt; jj += 256) {
    double2 z = a.zpart[p * nt + jj];
    for (int g = 1; g < a.S; ++g) z = c_add(z, a.zpart[((int64_t)g * a.n + p) * nt + jj]);
    buf[jj] = z;
  }
  tg_epilogue<HET>(a, p, buf, sm, sinv, red, red2);
}

gw_status tgrid_tables(gw_ctx* ctx, int L, int jmax, int K) {
  if (ctx->tm_ccoef && ctx->tm_cc_L == L && ctx->tm_cc_jmax == jmax && ctx->tm_cc_K == K) return GW_OK;
  int D1, D2;
  if (!tgrid_plan(L, &D1, &D2)) return set_error(GW_ENOTSUP, "time marginal: transform length %d not supported", L);
  std::vector<double> h;
  tgrid_coefficients(L, jmax, K, &h);
  if (ctx->tm_ccoef) (void)hipFree(ctx->tm_ccoef);
  ctx->tm_ccoef = nullptr;
  ctx->tm_cc_L = 0;
  gw_status s = check_hip(hipMalloc((void**)&ctx->tm_ccoef, h.size() * sizeof(double)), "time-grid coefficients");
  if (s == GW_OK) s = check_hip(hipMemcpy(ctx->tm_ccoef, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice),
                                "time-grid coefficients");
  if (s != GW_OK) return s;
  ctx->tm_cc_L = L;
  ctx->tm_cc_jmax = jmax;
  ctx->tm_cc_K = K;
  return GW_OK;
}

// Rows per chunk: the moments of a chunk take at most 1 GiB.
int64_t tgrid_chunk_rows(int64_t n, int n_blk, int K) {
  const int64_t per_row = (int64_t)K * n_blk * 16;
  int64_t c = ((int64_t)1 << 30) / per_row;
  if (c < 64) c = 64;
  return n < c ? n : c;
}

template <int HET>
static void launch_tgrid_form(const TgKernelArgs& k, int D1, int nz, unsigned n, hipStream_t st) {
  const dim3 grid((unsigned)(k.S * kTgXcds * ((n + kTgXcds - 1) / kTgXcds))), blk(256);
  switch (D1) {
    case 16:
      switch (nz) {
        case 1: hipLaunchKernelGGL((k_tgrid<HET, 16, 1>), grid, blk, 0, st, k); break;
        case 2: hipLaunchKernelGGL((k_tgrid<HET, 16, 2>), grid, blk, 0, st, k); break;
        case 4: hipLaunchKernelGGL((k_tgrid<HET, 16, 4>), grid, blk, 0, st, k); break;
        case 8: hipLaunchKernelGGL((k_tgrid<HET, 16, 8>), grid, blk, 0, st, k); break;
        default: hipLaunchKernelGGL((k_tgrid<HET, 16, 16>), grid, blk, 0, st, k); break;
      }
      break;
    case 8: hipLaunchKernelGGL((k_tgrid<HET, 8, 8>), grid, blk, 0, st, k); break;
    case 4: hipLaunchKernelGGL((k_tgrid<HET, 4, 4>), grid, blk, 0, st, k); break;
    case 2: hipLaunchKernelGGL((k_tgrid<HET, 2, 2>), grid, blk, 0, st, k); break;
    default: hipLaunchKernelGGL((k_tgrid<HET, 1, 1>), grid, blk, 0, st, k); break;
  }
  if (k.S > 1) hipLaunchKernelGGL((k_tgrid_fin<HET>), dim3(n), blk, 0, st, k);
}

// Order groups per row: a launch of few rows (a sampler round) would leave
// most of the 256 CUs idle with one workgroup per row, so its orders are
// split over 2 or 4 workgroups, whose partial sums k_tgrid_fin adds.
int tgrid_split(int64_t n, int K) {
  if (n >= 512) return 1;
  if (n >= 256 || K % 4 != 0) return K % 2 == 0 ? 2 : 1;
  return 4;
}

int64_t tgrid_zpart_elems(int64_t n, int64_t chunk, int K, int nt) {
  int64_t need = 0;
  for (const int64_t cn : {n < chunk ? n : chunk, n % chunk}) {  // full chunks and the last one
    const int S = tgrid_split(cn, K);
    if (cn > 0 && S > 1) need = std::max(need, (int64_t)S * cn * nt);
  }
  return need;
}

gw_status launch_tgrid(const gw_ctx* ctx, const TGridArgs& a, hipStream_t st) {
  int D1, D2;
  if (!tgrid_plan(a.L, &D1, &D2) || 2 * a.jmax + 1 > a.L)
    return set_error(GW_ENOTSUP, "time marginal: a grid of %d points per %d-point transform is not supported",
                     2 * a.jmax + 1, a.L);
  if (a.het && a.mh > kTgHMax) return set_error(GW_ENOTSUP, "time marginal: %d norm moments exceed %d", a.mh, kTgHMax);
  if (!ctx->tm_ccoef || ctx->tm_cc_L != a.L || ctx->tm_cc_jmax != a.jmax || ctx->tm_cc_K != a.K)
    return set_error(GW_ESTATE, "time marginal: coefficient table not built for this grid");
  if (a.n_blk > a.L) return set_error(GW_EINVAL, "time marginal: %d blocks exceed the transform length", a.n_blk);
  if (a.n <= 0) return GW_OK;
  // nonzero first-pass inputs per lane: blocks b = lane + (L / D1) q < n_blk
  const int S1 = a.L / D1;
  int nz = D1;
  if (D1 == 16) {
    const int need = (a.n_blk + S1 - 1) / S1;
    nz = 1;
    while (nz < need) nz <<= 1;
  }
  TgKernelArgs k{};
  k.mom = (const double2*)a.mom;
  k.mom_rs = a.mom_rs;
  k.mom_es = a.mom_es;
  k.n = a.n;
  k.n_blk = a.n_blk;
  k.L = a.L;
  k.D2 = D2;
  k.K = a.K;
  k.jmax = a.jmax;
  k.ccoef = ctx->tm_ccoef;
  k.coef = a.coef;
  k.ld = a.ld;
  k.dd = ctx->dd;
  k.logl = a.logl;
  k.zout = a.zout;
  k.f0_num = a.f0_num;
  k.f0_den = a.f0_den;
  k.cden = 1;
  k.S = tgrid_split(a.n, a.K);
  k.zpart = (double2*)a.zpart;
  if (k.S > 1 && !k.zpart) return set_error(GW_EINVAL, "time marginal: no workspace for the order groups");
  if (a.het) {
    k.hhc = a.hhc;
    k.hpart = (const double2*)a.hpart;
    k.n_hch = a.n_hch;
    k.mh = a.mh;
    k.hw_step = a.hw_step;
    k.c2 = a.c2;
    k.cden = a.cden;
    launch_tgrid_form<1>(k, D1, nz, (unsigned)a.n, st);
  } else {
    launch_tgrid_form<0>(k, D1, nz, (unsigned)a.n, st);
  }
  return check_hip(hipGetLastError(), "time-grid launch");
}

}  // namespace gw
