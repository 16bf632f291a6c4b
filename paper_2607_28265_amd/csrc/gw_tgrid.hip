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
// With M_bm = sum_{k in block b} s_k^m y_k (y the per-bin overlap weights of
// the full band, or the per-edge weights of the heterodyned bins),
//   Z(t_j) = exp(-2 pi i f_0 t_j) sum_{m < 16} (-i phi_j)^m / m! F_m(j),
//   F_m(j) = sum_b M_bm exp(-2 pi i b j / L),
// one length-L DFT per moment (16 terms leave a first dropped term below
// 1e-10 of the block's sum of |y|).  The leading factor has unit modulus.
//
// k_tgrid: one workgroup (256 lanes) per row.  For m = 15 .. 0 it runs a
// Stockham FFT of length L <= 4096 in radix-16 (then 8, 4 or 2) passes: the
// first pass reads the moments straight from memory (blocks beyond n_blk are
// zero), the others go through one LDS buffer of L values, at most one
// butterfly per lane and pass; each lane keeps the Horner recurrence over m
// for its own grid points.  Then ln I0(|Z|) - <h|h>(t_j) / 2 and a fixed-order
// log-sum-exp.  For the heterodyned bins the norm also depends on t_j:
// <h|h>(t_j) = hhc + Re exp(-2 pi i c u_j) sum_{m < MH} (-i x_j)^m / m! S_m,
// u_j = j / (N R) (fine-grid cycles), x_j = 2 pi hw u_j, with the bin widths
// dk_e = c + hw sigma_e expanded about their centre c and S_m the per-row
// moments sum_e sigma_e^m V_e (partial sums over edge chunks, added here in
// chunk order).
#include <math.h>

#include <vector>

#include "gw_ctx.h"
#include "gw_fft.h"

namespace gw {

constexpr int kTgMaxL = 4096;
constexpr int kTgOwn = 16;  // grid points per lane: 256 * 16 >= 2 jmax + 1 for L <= 4096

// One Stockham pass of radix R over buf (L points, span ns), at most one
// butterfly per lane; reads, waits, then writes in place.
template <int R>
__device__ inline void tg_pass(double2* __restrict__ buf, const double2* __restrict__ tw, int L, int ns, int tid) {
  const int nb = L / R;
  double2 v[R];
  const bool on = tid < nb;
  const int k = tid & (ns - 1);
  if (on) {
    const int stp = L / (ns * R);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      v[q] = buf[tid + q * nb];
      if (q > 0 && ns > 1) v[q] = c_mul(v[q], tw[k * q * stp]);
    }
  }
  __syncthreads();
  if (on) {
    Dft<R>::run_slots(v);
    const int base = (tid - k) * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) buf[base + q * ns] = v[dft_slot<R>(q)];
  }
  __syncthreads();
}

// First pass (span 1): inputs straight from the row's moments of order m.
template <int R>
__device__ inline void tg_first(double2* __restrict__ buf, const double2* __restrict__ src, int n_blk, int L,
                                int tid) {
  const int nb = L / R;
  if (tid < nb) {
    double2 v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int b = tid + q * nb;
      v[q] = b < n_blk ? src[b] : make_double2(0.0, 0.0);
    }
    Dft<R>::run_slots(v);
#pragma unroll
    for (int q = 0; q < R; ++q) buf[tid * R + q] = v[dft_slot<R>(q)];
  }
  __syncthreads();
}

__device__ inline void tg_run_first(int R, double2* buf, const double2* src, int n_blk, int L, int tid) {
  switch (R) {
    case 16: tg_first<16>(buf, src, n_blk, L, tid); break;
    case 8: tg_first<8>(buf, src, n_blk, L, tid); break;
    case 4: tg_first<4>(buf, src, n_blk, L, tid); break;
    default: tg_first<2>(buf, src, n_blk, L, tid); break;
  }
}

__device__ inline void tg_run_pass(int R, double2* buf, const double2* tw, int L, int ns, int tid) {
  switch (R) {
    case 16: tg_pass<16>(buf, tw, L, ns, tid); break;
    case 8: tg_pass<8>(buf, tw, L, ns, tid); break;
    case 4: tg_pass<4>(buf, tw, L, ns, tid); break;
    default: tg_pass<2>(buf, tw, L, ns, tid); break;
  }
}

// mom: [n][16][n_blk] complex (row p, order m, block b at ((p 16 + m) n_blk + b)).
// HET = 0: <h|h> = coef[C_HH]; HET = 1: <h|h>(t_j) as above from hhc [n], the
// H moments hpart [n_hch][n][mh] complex, hw_step = 2 pi hw / (N R), c2 = 2 c
// and cden = 2 N R (exp(-2 pi i c u_j) = exp(-2 pi i (c2 j mod cden) / cden)).
// zout (else NULL): [n][2 jmax + 1][3] = (Re Z(t_j), Im Z(t_j), <h|h>(t_j)),
// Re NaN for unphysical rows, with f_0 t_j = j f0_num / f0_den cycles.
template <int HET>
__global__ void __launch_bounds__(256, 2) k_tgrid(const double2* __restrict__ mom, int64_t n, int n_blk, int L,
                                               int4 radix, int n_pass, const double2* __restrict__ tw, int jmax,
                                               double phi_step, const double* __restrict__ coef, int64_t ld, double dd,
                                               const LogI0Consts* __restrict__ Cp, double* __restrict__ logl,
                                               const double* __restrict__ hhc, const double2* __restrict__ hpart,
                                               int n_hch, int mh, double hw_step, int64_t c2, int64_t cden,
                                               double* __restrict__ zout, double f0_num, double f0_den) {
  __shared__ double2 buf[kTgMaxL];
  __shared__ double2 sm[kTgHMax];
  __shared__ double red[256], red2[256];
  const int64_t p = blockIdx.x;
  const int tid = threadIdx.x;
  const int nt = 2 * jmax + 1;
  const int rad[4] = {radix.x, radix.y, radix.z, radix.w};
  double ar[kTgOwn], ai[kTgOwn];
#pragma unroll
  for (int o = 0; o < kTgOwn; ++o) ar[o] = ai[o] = 0.0;
  for (int m = kTMomOrders - 1; m >= 0; --m) {
    __syncthreads();  // the previous order's grid reads are done
    tg_run_first(rad[0], buf, mom + (p * kTMomOrders + m) * n_blk, n_blk, L, tid);
    int ns = rad[0];
    for (int s = 1; s < n_pass; ++s) {
      tg_run_pass(rad[s], buf, tw, L, ns, tid);
      ns *= rad[s];
    }
    // H = F_m + (-i phi_j / (m + 1)) H at this lane's grid points
    const double inv = phi_step / (double)(m + 1);
#pragma unroll
    for (int o = 0; o < kTgOwn; ++o) {
      const int jj = tid + 256 * o;
      if (jj < nt) {
        const int j = jj - jmax;
        const double2 f = buf[j < 0 ? j + L : j];
        const double qq = inv * (double)j;
        const double nr = fma(qq, ai[o], f.x), ni = fma(-qq, ar[o], f.y);
        ar[o] = nr;
        ai[o] = ni;
      }
    }
  }
  const bool valid = coef[C_VALID * ld + p] != 0.0;
  const LogI0Consts& C = *Cp;
  // the finished Z(t_j) go to the buffer (nt <= L points), read back below
  // in a plain loop
  __syncthreads();
#pragma unroll
  for (int o = 0; o < kTgOwn; ++o) {
    const int jj = tid + 256 * o;
    if (jj < nt) buf[jj] = make_double2(ar[o], ai[o]);
  }
  double hh = 0.0;
  if (HET) {
    hh = hhc[p];
    // this row's H moments, summed over the edge chunks in order
    for (int q = tid; q < mh; q += 256) {
      double2 a = make_double2(0.0, 0.0);
      for (int c = 0; c < n_hch; ++c) a = c_add(a, hpart[((int64_t)c * n + p) * mh + q]);
      sm[q] = a;
    }
  } else {
    hh = coef[C_HH * ld + p];
  }
  __syncthreads();
  double run_mx = -INFINITY, run_acc = 0.0;
  for (int jj = tid; jj < nt; jj += 256) {
    const int j = jj - jmax;
    const double2 z = buf[jj];
    double hj = hh;
    if (HET) {
      const double x = hw_step * (double)j;
      double tr = 0.0, ti = 0.0;
      for (int q = mh - 1; q >= 0; --q) {
        const double qq = x / (double)(q + 1);
        const double nr = fma(qq, ti, sm[q].x), ni = fma(-qq, tr, sm[q].y);
        tr = nr;
        ti = ni;
      }
      const int64_t num = (c2 * (int64_t)j) % cden;
      double sn, cs;
      sincospi(-2.0 * (double)num / (double)cden, &sn, &cs);
      hj += cs * tr - sn * ti;
    }
    if (zout) {
      const double cyc = (double)j * f0_num / f0_den;
      double sn, cs;
      sincospi(2.0 * (cyc - rint(cyc)), &sn, &cs);
      double* zo = zout + (p * nt + jj) * 3;
      zo[0] = valid ? cs * z.x + sn * z.y : NAN;
      zo[1] = cs * z.y - sn * z.x;
      zo[2] = hj;
    }
    const double v = -0.5 * hj + log_i0(sqrt(z.x * z.x + z.y * z.y), C);
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
  if (tid == 0) logl[p] = valid ? -0.5 * dd + red[0] + log(red2[0]) - log((double)nt) : -INFINITY;
}

// Radix plan for a length L = 2^q <= 4096: radix-16 passes, then one of 8, 4
// or 2 for the rest (at most one butterfly per lane of 256 in every pass).
bool tgrid_plan(int L, int4* radix, int* n_pass) {
  if (L < 2 || L > kTgMaxL || (L & (L - 1)) != 0) return false;
  int r[4] = {0, 0, 0, 0};
  int np = 0, rest = L;
  while (rest >= 16) {
    r[np++] = 16;
    rest /= 16;
  }
  if (rest > 1) r[np++] = rest;
  *radix = make_int4(r[0], r[1], r[2], r[3]);
  *n_pass = np;
  return true;
}

gw_status tgrid_twiddles(gw_ctx* ctx, int L) {
  if (ctx->tm_tw && ctx->tm_L == L) return GW_OK;
  std::vector<double> h(2 * (size_t)L);
  for (int t = 0; t < L; ++t) {
    const double a = -2.0 * kPi * (double)t / (double)L;
    h[2 * t] = cos(a);
    h[2 * t + 1] = sin(a);
  }
  if (ctx->tm_tw) (void)hipFree(ctx->tm_tw);
  ctx->tm_tw = nullptr;
  ctx->tm_L = 0;
  gw_status s = check_hip(hipMalloc((void**)&ctx->tm_tw, h.size() * sizeof(double)), "time-grid twiddles");
  if (s == GW_OK) s = check_hip(hipMemcpy(ctx->tm_tw, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice),
                                "time-grid twiddles");
  if (s == GW_OK) ctx->tm_L = L;
  return s;
}

// Rows per chunk: the moments of a chunk take at most 1 GiB.
int64_t tgrid_chunk_rows(int64_t n, int n_blk) {
  const int64_t per_row = (int64_t)kTMomOrders * n_blk * 16;
  int64_t c = ((int64_t)1 << 30) / per_row;
  if (c < 64) c = 64;
  return n < c ? n : c;
}

gw_status launch_tgrid(const gw_ctx* ctx, const TGridArgs& a, hipStream_t st) {
  int4 radix;
  int n_pass;
  if (!tgrid_plan(a.L, &radix, &n_pass) || 2 * a.jmax + 1 > 256 * kTgOwn)
    return set_error(GW_ENOTSUP, "time marginal: a grid of %d points per %d-point transform is not supported",
                     2 * a.jmax + 1, a.L);
  if (a.het && a.mh > kTgHMax) return set_error(GW_ENOTSUP, "time marginal: %d norm moments exceed %d", a.mh, kTgHMax);
  const double phi_step = kPi / (double)a.L;
  const LogI0Consts* C = ctx->i0c;
  if (a.het)
    hipLaunchKernelGGL(k_tgrid<1>, dim3((unsigned)a.n), dim3(256), 0, st, (const double2*)a.mom, a.n, a.n_blk, a.L,
                       radix, n_pass, (const double2*)a.tw, a.jmax, phi_step, a.coef, a.ld, ctx->dd, C, a.logl,
                       a.hhc, (const double2*)a.hpart, a.n_hch, a.mh, a.hw_step, a.c2, a.cden, a.zout, a.f0_num,
                       a.f0_den);
  else
    hipLaunchKernelGGL(k_tgrid<0>, dim3((unsigned)a.n), dim3(256), 0, st, (const double2*)a.mom, a.n, a.n_blk, a.L,
                       radix, n_pass, (const double2*)a.tw, a.jmax, phi_step, a.coef, a.ld, ctx->dd, C, a.logl,
                       nullptr, nullptr, 0, 0, 0.0, (int64_t)0, (int64_t)1, a.zout, a.f0_num, a.f0_den);
  return check_hip(hipGetLastError(), "time-grid launch");
}

}  // namespace gw
