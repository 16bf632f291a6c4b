// Coalescence-time marginal on the full band (Sec. III.A and the appendix on
// grid marginalisations: a log-sum-exp over a grid of time shifts, computed
// by FFT on the uniform grid), together with the phase marginal.
//
// Grid: t_j = j delta, |j| <= J = floor(W / delta), delta = 1 / (N df) with N
// the smallest power of two >= 2 (k0 + n_freq - 1) (the segment's sampling
// interval).  With the template at t_c = 0,
//   log L = -<d|d>/2 - <h|h>/2 + ln[ (1 / (2J + 1)) sum_j I0(|Z(t_j)|) ],
//   Z(t)  = sum_k y_k exp(-2 pi i f_k t),
//   y_k   = 4 df sum_i d_ik* h_ik / S_ik = g_k sum_i (A P_i) u_ik exp(-2 pi i f_k dtau_i),
// g_k the detector-0 phasor (template phase including detector 0's delay) and
// dtau_i the other detectors' delays relative to detector 0.
//
// Evaluation.  P is the smallest power of two >= 2J + 1 and the band is cut
// into blocks of B = N / P bins, so that the block centres f_b = f_0 + b B df
// give exp(-2 pi i f_b t_j) = exp(-2 pi i f_0 t_j) w^(b j), w = exp(-2 pi i / P):
// a P-point DFT over blocks.  Inside a block, with s = (k - kb - (B-1)/2) / (B/2),
//   exp(-2 pi i f_k t_j) = exp(-2 pi i f_b t_j) exp(-i phi_j s),  phi_j = pi df B t_j,
// and |phi_j| <= pi J / P < pi / 2, so 16 terms of the exponential series
// (first dropped term below 1e-10 of the block's sum of |y|) give
//   Z(t_j) = exp(-2 pi i f_0 t_j) sum_m (-i phi_j)^m / m! DFT_b(M_bm)(j),
//   M_bm   = sum_{k in block b} s_k^m y_k.
// The leading factor has unit modulus, so |Z(t_j)| needs only the 16 DFTs.
//   k_tmom: per (proposal, block), the 16 moments M_bm (lane = proposal, the
//           workgroup's waves walk the same block, wave-uniform bin records
//           as in the full-band reduction);
//   k_tmarg: one workgroup per proposal: for m = 15 .. 0, a P-point radix-4
//           Stockham FFT of M_.m in LDS, folded into a Horner recurrence over
//           m for every owned grid point; then ln I0(|Z|) and a fixed-order
//           log-sum-exp.
#include <math.h>

#include <vector>

#include "gw_ctx.h"

namespace gw {

constexpr int kTMom = 16;
constexpr int kTMaxP = 2048;

template <int PREC>
__device__ inline void tm_phasor(double r, const TrigConsts& T, double* gr, double* gi) {
  if (PREC == 0) {
    double s, c;
    sincos_cycles(r, T, &s, &c);
    *gr = c;
    *gi = -s;
  } else {
    const float t = (float)(r - rint(r));
    *gr = (double)__builtin_amdgcn_cosf(t);
    *gi = -(double)__builtin_amdgcn_sinf(t);
  }
}

template <int ND, int PREC>
__global__ void __launch_bounds__(256) k_tmom(const double* __restrict__ coef, int64_t ld, int64_t n,
                                              const double* __restrict__ bins, int64_t k0, double df, int n_freq,
                                              int blk, int n_blk, TrigConsts T, double pg_re, double pg_im,
                                              const double* __restrict__ tpow, double* __restrict__ mom) {
  constexpr int RS = 4 + 2 * ND;
  const int tpb = blockDim.x;
  const int nptile = (int)((n + tpb - 1) / tpb);
  const int b = blockIdx.x / nptile, ptile = blockIdx.x - b * nptile;
  const int64_t p = (int64_t)ptile * tpb + threadIdx.x;
  const int64_t pc = p < n ? p : n - 1;

  PhaseCoef c;
  c.a0 = coef[C_A0 * ld + pc];
  c.a2 = coef[C_A2 * ld + pc];
  c.a3 = coef[C_A3 * ld + pc];
  c.a4 = coef[C_A4 * ld + pc];
  c.a5 = coef[C_A5 * ld + pc];
  c.a6 = coef[C_A6 * ld + pc];
  c.a7 = coef[C_A7 * ld + pc];
  c.a8 = coef[C_A8 * ld + pc];
  c.a10 = coef[C_A10 * ld + pc];
  c.a12 = coef[C_A12 * ld + pc];
  c.b5 = coef[C_B5 * ld + pc];
  c.b6 = coef[C_B6 * ld + pc];
  // e_i = (A P_i) exp(-2 pi i f_k dtau_i), advanced bin by bin by the rotation
  // rho_i = exp(-2 pi i df dtau_i) (detector 0: the constant A P_0)
  double er[ND], ei[ND], rr[ND], ri[ND];
  const int kb = b * blk;
  const int ke = kb + blk < n_freq ? kb + blk : n_freq;
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    const double apr = coef[(C_APRE + i) * ld + pc], api = coef[(C_APIM + i) * ld + pc];
    er[i] = apr;
    ei[i] = api;
    rr[i] = 1.0;
    ri[i] = 0.0;
    if (i > 0) {
      const double dt = coef[(C_DT1 + i - 1) * ld + pc];
      double s, co;
      sincos_cycles((double)(k0 + kb) * df * dt, T, &s, &co);
      er[i] = apr * co + api * s;
      ei[i] = api * co - apr * s;
      sincos_cycles(df * dt, T, &s, &co);
      rr[i] = co;
      ri[i] = -s;
    }
  }
  double mr[kTMom], mi[kTMom];
#pragma unroll
  for (int m = 0; m < kTMom; ++m) mr[m] = mi[m] = 0.0;
  for (int k = kb; k < ke; ++k) {
    const double* __restrict__ rec = bins + (int64_t)k * RS;
    const double r = phase_cycles(c, rec[0], rec[1], rec[2], rec[3]);
    double gr, gi;
    tm_phasor<PREC>(r, T, &gr, &gi);
    // s = sum_i u_ik e_i
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const double ur = rec[4 + 2 * i], ui = rec[5 + 2 * i];
      sr = fma(ur, er[i], sr);
      sr = fma(-ui, ei[i], sr);
      si = fma(ur, ei[i], si);
      si = fma(ui, er[i], si);
      if (i > 0) {
        const double tr = er[i] * rr[i] - ei[i] * ri[i];
        ei[i] = er[i] * ri[i] + ei[i] * rr[i];
        er[i] = tr;
      }
    }
    const double yr = gr * sr - gi * si, yi = gr * si + gi * sr;
    // the powers t^m of the bin's offset in the block come from a table
    // (the same for every block and proposal: wave-uniform scalar loads)
    const double* __restrict__ tq = tpow + (int64_t)(k - kb) * kTMom;
#pragma unroll
    for (int m = 0; m < kTMom; ++m) {
      mr[m] = fma(tq[m], yr, mr[m]);
      mi[m] = fma(tq[m], yi, mi[m]);
    }
  }
  if (p >= n) return;
  double* __restrict__ out = mom + (p * kTMom * n_blk + b) * 2;
#pragma unroll
  for (int m = 0; m < kTMom; ++m) {
    double vr = mr[m], vi = mi[m];
    if (PREC == 1) {  // remove the mean bias of the hardware phasor
      const double tr = vr * pg_re - vi * pg_im;
      vi = vr * pg_im + vi * pg_re;
      vr = tr;
    }
    out[(int64_t)m * n_blk * 2] = vr;
    out[(int64_t)m * n_blk * 2 + 1] = vi;
  }
}

// One workgroup (256 threads) per proposal; P <= kTMaxP.  Dynamic LDS: two
// buffers of P complex values.
// The grid is oversampled R times: sub-grid r holds t = (j + r / R) delta,
// |j| <= J for r = 0 and -J <= j < J otherwise (2 J R + 1 points in all).  A
// shift of r delta / R multiplies block b's term by exp(-2 pi i b r / (R P))
// (``sh`` [R][P]), applied to the moments before the FFT.  The log-sum-exp runs
// over every point of every sub-grid, in a fixed order.
// With zout (else NULL) each row's grid values are also staged for post-hoc
// draws: zout[p][i] = (Re Z(t_i), Im Z(t_i), <h|h>), t_i = (i - J R) delta / R
// (Re NaN for unphysical rows), the unit factor exp(-2 pi i f_0 t_i) restored:
// f_0 t_i = (i - J R) f0_num / (f0_den R) cycles exactly, f0_num = 2 k0 + B - 1
// and f0_den = 2 N.
__global__ void __launch_bounds__(256) k_tmarg(const double* __restrict__ mom, int64_t n, int n_blk, int P, int J,
                                               int R, const double2* __restrict__ tw, const double2* __restrict__ sh,
                                               double phi_step, const double* __restrict__ coef, int64_t ld,
                                               double dd, LogI0Consts C, double* __restrict__ logl,
                                               double* __restrict__ zout, double f0_num, double f0_den) {
  extern __shared__ double2 lds_fft[];
  double2* buf[2] = {lds_fft, lds_fft + P};
  __shared__ double red[256];
  constexpr int kOwn = kTMaxP / 256;  // grid points per thread and sub-grid (at most)
  const int64_t p = blockIdx.x;
  const int tid = threadIdx.x;
  const int nj = 2 * J + 1;
  const int nt = 2 * J * R + 1;
  const bool valid = coef[C_VALID * ld + p] != 0.0;
  const double hh = coef[C_HH * ld + p];
  double run_mx = -INFINITY, run_acc = 0.0;  // this thread's log-sum-exp so far
  for (int r = 0; r < R; ++r) {
    const double frac = (double)r / (double)R;
    double hr[kOwn], hi[kOwn];
#pragma unroll
    for (int q = 0; q < kOwn; ++q) hr[q] = hi[q] = 0.0;
    for (int m = kTMom - 1; m >= 0; --m) {
      const double* __restrict__ src = mom + (p * kTMom + m) * n_blk * 2;
      for (int b = tid; b < P; b += 256) {
        double2 v = b < n_blk ? make_double2(src[2 * b], src[2 * b + 1]) : make_double2(0.0, 0.0);
        if (r > 0) {
          const double2 w = sh[r * P + b];
          v = make_double2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
        }
        buf[0][b] = v;
      }
      __syncthreads();
      // Stockham FFT: radix-4 stages while they fit, then one radix-2 stage
      // when log2 P is odd (twiddles w^t = exp(-2 pi i t / P), t < P / 2)
      int cur = 0;
      for (int ns = 1; ns < P;) {
        const double2* __restrict__ src = buf[cur];
        double2* __restrict__ dst = buf[cur ^ 1];
        if (4 * ns <= P) {
          const int q4 = P / 4, stp = P / (4 * ns);
          for (int j = tid; j < q4; j += 256) {
            const int k = j & (ns - 1);
            const double2 w1 = tw[k * stp], w2 = tw[2 * k * stp];
            const double2 w3 = make_double2(w1.x * w2.x - w1.y * w2.y, w1.x * w2.y + w1.y * w2.x);
            const double2 a0 = src[j];
            const double2 x1 = src[j + q4], x2 = src[j + 2 * q4], x3 = src[j + 3 * q4];
            const double2 a1 = make_double2(x1.x * w1.x - x1.y * w1.y, x1.x * w1.y + x1.y * w1.x);
            const double2 a2 = make_double2(x2.x * w2.x - x2.y * w2.y, x2.x * w2.y + x2.y * w2.x);
            const double2 a3 = make_double2(x3.x * w3.x - x3.y * w3.y, x3.x * w3.y + x3.y * w3.x);
            const double2 b0 = make_double2(a0.x + a2.x, a0.y + a2.y), b1 = make_double2(a0.x - a2.x, a0.y - a2.y);
            const double2 b2 = make_double2(a1.x + a3.x, a1.y + a3.y);
            const double2 b3 = make_double2(a1.y - a3.y, a3.x - a1.x);  // (a1 - a3) (-i)
            const int idx = ((j - k) << 2) + k;
            dst[idx] = make_double2(b0.x + b2.x, b0.y + b2.y);
            dst[idx + ns] = make_double2(b1.x + b3.x, b1.y + b3.y);
            dst[idx + 2 * ns] = make_double2(b0.x - b2.x, b0.y - b2.y);
            dst[idx + 3 * ns] = make_double2(b1.x - b3.x, b1.y - b3.y);
          }
          ns *= 4;
        } else {
          for (int j = tid; j < P / 2; j += 256) {
            const double2 v0 = src[j];
            const double2 x1 = src[j + P / 2];
            const int k = j & (ns - 1);
            const double2 w = tw[k * (P / (2 * ns))];
            const double v1r = x1.x * w.x - x1.y * w.y, v1i = x1.x * w.y + x1.y * w.x;
            const int idx = ((j - k) << 1) + k;
            dst[idx] = make_double2(v0.x + v1r, v0.y + v1i);
            dst[idx + ns] = make_double2(v0.x - v1r, v0.y - v1i);
          }
          ns *= 2;
        }
        __syncthreads();
        cur ^= 1;
      }
      // H = F_m + (-i phi(t) / (m + 1)) H, phi(t) = phi_step (j + r / R)
      const double inv = 1.0 / (double)(m + 1);
#pragma unroll
      for (int q = 0; q < kOwn; ++q) {
        const int jj = tid + 256 * q;
        if (jj < nj) {
          const int j = jj - J;
          const double2 f = buf[cur][j < 0 ? j + P : j];
          const double qq = phi_step * ((double)j + frac) * inv;
          const double nr = fma(qq, hi[q], f.x), ni = fma(-qq, hr[q], f.y);
          hr[q] = nr;
          hi[q] = ni;
        }
      }
      __syncthreads();  // before the next moment overwrites the buffers
    }
#pragma unroll
    for (int q = 0; q < kOwn; ++q) {
      const int jj = tid + 256 * q;
      if (jj >= nj || (r > 0 && jj == nj - 1)) continue;  // sub-grids r > 0 stop one step short
      const int i = jj * R + r;                               // position on the full grid
      if (zout) {
        const double cyc = (double)(i - J * R) * f0_num / (f0_den * (double)R);
        double sn, cs;
        sincospi(2.0 * (cyc - rint(cyc)), &sn, &cs);
        double* o = zout + (p * nt + i) * 3;
        o[0] = valid ? cs * hr[q] + sn * hi[q] : NAN;
        o[1] = cs * hi[q] - sn * hr[q];
        o[2] = hh;
      }
      const double v = log_i0(sqrt(hr[q] * hr[q] + hi[q] * hi[q]), C);
      if (v > run_mx) {
        run_acc = run_acc * exp(run_mx - v) + 1.0;
        run_mx = v;
      } else {
        run_acc += exp(v - run_mx);
      }
    }
  }
  red[tid] = run_mx;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (tid < s2) red[tid] = fmax(red[tid], red[tid + s2]);
    __syncthreads();
  }
  const double ref = red[0];
  __syncthreads();
  red[tid] = run_acc > 0.0 ? run_acc * exp(run_mx - ref) : 0.0;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (tid < s2) red[tid] += red[tid + s2];
    __syncthreads();
  }
  if (tid == 0) logl[p] = valid ? -0.5 * dd - 0.5 * hh + ref + log(red[0]) - log((double)nt) : -INFINITY;
}

template <int ND>
static void launch_tmom_nd(gw_ctx* ctx, const double* coef, int64_t n, int prec, int blk, int n_blk, int tpb,
                           double* mom, hipStream_t st) {
  const int64_t nptile = (n + tpb - 1) / tpb;
  const TrigConsts T = make_trig_consts();
  if (prec == GW_PREC_FP64)
    hipLaunchKernelGGL((k_tmom<ND, 0>), dim3((unsigned)(nptile * n_blk)), dim3(tpb), 0, st, coef, n, n, ctx->bins,
                       ctx->geom.k0, ctx->geom.df, (int)ctx->geom.n_freq, blk, n_blk, T, 1.0, 0.0,
                       (const double*)ctx->tm_tpow, mom);
  else
    hipLaunchKernelGGL((k_tmom<ND, 1>), dim3((unsigned)(nptile * n_blk)), dim3(tpb), 0, st, coef, n, n, ctx->bins,
                       ctx->geom.k0, ctx->geom.df, (int)ctx->geom.n_freq, blk, n_blk, T, ctx->pgain_re,
                       ctx->pgain_im, (const double*)ctx->tm_tpow, mom);
}

// Grid of the time marginal for the context's window: N, J, P, B.
struct TimeGrid {
  int64_t N;
  double delta;  // the segment's sampling interval; the grid step is delta / R
  int J, R, P, blk, n_blk;
};

static gw_status time_grid(const gw_ctx* ctx, TimeGrid* g) {
  const int64_t top = 2 * (ctx->geom.k0 + ctx->geom.n_freq - 1);
  int64_t N = 1;
  while (N < top) N <<= 1;
  g->N = N;
  g->delta = 1.0 / ((double)N * ctx->geom.df);
  g->J = (int)floor(ctx->tm_window / g->delta + 1e-9);
  g->R = ctx->tm_R;
  int P = 2;
  while (P < 2 * g->J + 1) P <<= 1;
  if (P > kTMaxP) return set_error(GW_ENOTSUP, "time marginal: window %.6g s needs more than %d grid points",
                                   ctx->tm_window, kTMaxP);
  if (N / P < 1) return set_error(GW_ENOTSUP, "time marginal: grid finer than the segment's sampling");
  g->P = P;
  g->blk = (int)(N / P);
  g->n_blk = (int)((ctx->geom.n_freq + g->blk - 1) / g->blk);
  return GW_OK;
}

gw_status loglike_tmarg(gw_ctx* ctx, const double* theta, int64_t n, int prec, double* logl, hipStream_t st) {
  return loglike_tmarg_staged(ctx, theta, n, prec, logl, nullptr, st);
}

gw_status loglike_tmarg_staged(gw_ctx* ctx, const double* theta, int64_t n, int prec, double* logl, double* zout,
                               hipStream_t st) {
  TimeGrid g;
  gw_status s = time_grid(ctx, &g);
  if (s != GW_OK) return s;
  if (ctx->tm_P != g.P || ctx->tm_twR != g.R) {
    // twiddles w^k = exp(-2 pi i k / P), k < P / 2, then the sub-grid shifts
    // exp(-2 pi i b r / (R P)) [R][P], in FP64
    std::vector<double> h((size_t)g.P + 2 * (size_t)g.R * g.P);
    for (int k = 0; k < g.P / 2; ++k) {
      const double a = -2.0 * kPi * (double)k / (double)g.P;
      h[2 * k] = cos(a);
      h[2 * k + 1] = sin(a);
    }
    for (int r = 0; r < g.R; ++r)
      for (int b = 0; b < g.P; ++b) {
        const double a = -2.0 * kPi * (double)((int64_t)b * r) / ((double)g.R * g.P);
        h[g.P + 2 * ((size_t)r * g.P + b)] = cos(a);
        h[g.P + 2 * ((size_t)r * g.P + b) + 1] = sin(a);
      }
    if (ctx->tm_tw) (void)hipFree(ctx->tm_tw);
    ctx->tm_tw = nullptr;
    ctx->tm_P = 0;
    s = check_hip(hipMalloc((void**)&ctx->tm_tw, h.size() * sizeof(double)), "time-grid twiddles");
    if (s == GW_OK)
      s = check_hip(hipMemcpy(ctx->tm_tw, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice), "twiddles");
    if (s != GW_OK) return s;
    ctx->tm_P = g.P;
    ctx->tm_twR = g.R;
  }
  if (ctx->tm_tpow_blk != g.blk) {
    // powers t_j^m, t_j = (j - (B - 1) / 2) / (B / 2), m < 16, formed as the
    // moment sums use them (repeated products from 1)
    std::vector<double> h((size_t)g.blk * kTMom);
    const double cen = 0.5 * (g.blk - 1), hinv = 2.0 / g.blk;
    for (int j = 0; j < g.blk; ++j) {
      const double t = ((double)j - cen) * hinv;
      double tp = 1.0;
      for (int m = 0; m < kTMom; ++m) {
        h[(size_t)j * kTMom + m] = tp;
        tp *= t;
      }
    }
    if (ctx->tm_tpow) (void)hipFree(ctx->tm_tpow);
    ctx->tm_tpow = nullptr;
    ctx->tm_tpow_blk = 0;
    s = check_hip(hipMalloc((void**)&ctx->tm_tpow, h.size() * sizeof(double)), "time-grid powers");
    if (s == GW_OK)
      s = check_hip(hipMemcpy(ctx->tm_tpow, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice), "powers");
    if (s != GW_OK) return s;
    ctx->tm_tpow_blk = g.blk;
  }
  s = ensure_buffer(&ctx->coef, &ctx->coef_cap, (int64_t)C_NCOEF * n, "coefficient workspace");
  if (s == GW_OK) s = ensure_buffer(&ctx->tm_mom, &ctx->tm_mom_cap, n * kTMom * g.n_blk * 2, "time moments");
  if (s != GW_OK) return s;
  s = launch_prologue(ctx, theta, n, GW_MARG_PHASE_TIME, ctx->coef, n, st);
  if (s != GW_OK) return s;
  const int tpb = n >= 2048 ? 256 : 64;
  const int slot = prof_begin(ctx, st);
  switch (ctx->n_det) {
    case 1: launch_tmom_nd<1>(ctx, ctx->coef, n, prec, g.blk, g.n_blk, tpb, ctx->tm_mom, st); break;
    case 2: launch_tmom_nd<2>(ctx, ctx->coef, n, prec, g.blk, g.n_blk, tpb, ctx->tm_mom, st); break;
    case 3: launch_tmom_nd<3>(ctx, ctx->coef, n, prec, g.blk, g.n_blk, tpb, ctx->tm_mom, st); break;
    case 4: launch_tmom_nd<4>(ctx, ctx->coef, n, prec, g.blk, g.n_blk, tpb, ctx->tm_mom, st); break;
    default: return set_error(GW_ENOTSUP, "n_det %d not supported", ctx->n_det);
  }
  prof_end(ctx, slot, st);
  s = check_hip(hipGetLastError(), "time moments launch");
  if (s != GW_OK) return s;
  LogI0Consts C = make_log_i0_consts();
  C.r1max = ctx->dist_r1max;
  const double phi_step = kPi * ctx->geom.df * g.blk * g.delta;
  hipLaunchKernelGGL(k_tmarg, dim3((unsigned)n), dim3(256), 2 * g.P * sizeof(double2), st,
                     (const double*)ctx->tm_mom, n, g.n_blk, g.P, g.J, g.R, (const double2*)ctx->tm_tw,
                     (const double2*)ctx->tm_tw + g.P / 2, phi_step, (const double*)ctx->coef, n, ctx->dd, C, logl,
                     zout, (double)(2 * ctx->geom.k0 + g.blk - 1), (double)(2 * g.N));
  return check_hip(hipGetLastError(), "time marginal launch");
}

}  // namespace gw

extern "C" gw_status gw_set_time_window(gw_ctx* ctx, double window) {
  if (!ctx) return gw::set_error(GW_EINVAL, "gw_set_time_window: ctx is NULL");
  if (!(window >= 0.0) || !isfinite(window)) return gw::set_error(GW_EINVAL, "gw_set_time_window: window >= 0");
  const double old = ctx->tm_window;
  ctx->tm_window = window;
  gw::TimeGrid g;
  const gw_status s = gw::time_grid(ctx, &g);
  if (s != GW_OK) ctx->tm_window = old;
  return s;
}

extern "C" gw_status gw_set_time_oversample(gw_ctx* ctx, int32_t factor) {
  if (!ctx) return gw::set_error(GW_EINVAL, "gw_set_time_oversample: ctx is NULL");
  if (factor != 1 && factor != 2 && factor != 4 && factor != 8 && factor != 16)
    return gw::set_error(GW_EINVAL, "gw_set_time_oversample: factor must be 1, 2, 4, 8 or 16");
  ctx->tm_R = factor;
  return GW_OK;
}

extern "C" gw_status gw_time_grid_info(const gw_ctx* ctx, double* delta, int32_t* n_points, int32_t* fft_len,
                                       int32_t* block_bins) {
  if (!ctx) return gw::set_error(GW_EINVAL, "gw_time_grid_info: ctx is NULL");
  gw::TimeGrid g;
  const gw_status s = gw::time_grid(ctx, &g);
  if (s != GW_OK) return s;
  if (delta) *delta = g.delta / g.R;
  if (n_points) *n_points = 2 * g.J * g.R + 1;
  if (fft_len) *fft_len = g.P;
  if (block_bins) *block_bins = g.blk;
  return GW_OK;
}
