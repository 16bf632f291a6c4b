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
// into blocks of B = N / P bins (512 at 128 s); the grid sum then goes through
// the block moments M_bm = sum_{k in block b} T_m(s_k) y_k of the projected
// data (T_m the Chebyshev polynomials, s_k the bin's offset in its block
// scaled to [-1, 1]) and one FFT of length P R per order (gw_tgrid.hip):
//   k_tmom:  per (proposal, block), the K moments (lane = proposal, the
//            workgroup's waves walk the same block, wave-uniform bin records
//            as in the full-band reduction);
//   k_tgrid: one workgroup per proposal, FFTs weighted by the expansion
//            coefficients, ln I0(|Z|) and a fixed-order log-sum-exp.
// Rows go through in chunks whose moments fit a bounded workspace.
#include <math.h>

#include <vector>

#include "gw_ctx.h"
#include "gw_phase.h"
#include "gw_tgrid.h"

namespace gw {

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

// Per (256-row tile, block): lane = row, the block's bins walked from the top
// down (wave-uniform records).  FP64: the phase of every bin by its full
// series.  Mixed: the phase by the cubic recurrence in the runs of the
// full-band walk (gw_phase.h: a bin's phase depends on its run alone, so it
// is the same here as in the distance-marginal reduction), FP32 hardware
// sin/cos, FP64 sums.
// e_i = (A P_i) exp(-2 pi i f_k dtau_i) starts at the block's top bin and
// steps down by conj(rho_i), rho_i = exp(-2 pi i df dtau_i).
template <int ND, int PREC, int K>
__global__ void __launch_bounds__(256) k_tmom(const double* __restrict__ coef, int64_t ld, int64_t n,
                                              const double* __restrict__ bins, int64_t k0, double df, int n_freq,
                                              int blk, int n_blk, TrigConsts T, PhaseRuns R, double pg_re,
                                              double pg_im, const double* __restrict__ basis,
                                              double* __restrict__ mom) {
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
  const int kb = b * blk;
  const int ke = kb + blk < n_freq ? kb + blk : n_freq;
  double er[ND], ei[ND], rr[ND], ri[ND];
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
      sincos_cycles((double)(k0 + ke - 1) * df * dt, T, &s, &co);
      er[i] = apr * co + api * s;
      ei[i] = api * co - apr * s;
      sincos_cycles(df * dt, T, &s, &co);
      rr[i] = co;
      ri[i] = s;  // conj(rho_i): the walk descends
    }
  }
  double mr[K], mi[K];
#pragma unroll
  for (int m = 0; m < K; ++m) mr[m] = mi[m] = 0.0;
  // one bin: y = g sum_i u_ik e_i into the moments, then e_i one bin down
  auto visit = [&](int k, double gr, double gi) {
    const double* __restrict__ u = bins + (int64_t)k * RS + 4;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const double ur = u[2 * i], ui = u[2 * i + 1];
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
    // T_m of the bin's offset in the block come from a table (the same for
    // every block and proposal: wave-uniform scalar loads)
    const double* __restrict__ tq = basis + (int64_t)(k - kb) * K;
#pragma unroll
    for (int m = 0; m < K; ++m) {
      mr[m] = fma(tq[m], yr, mr[m]);
      mi[m] = fma(tq[m], yi, mi[m]);
    }
  };
  if constexpr (PREC == 0) {
    for (int k = ke - 1; k >= kb; --k) {
      const double* __restrict__ rec = bins + (int64_t)k * RS;
      double gr, gi;
      tm_phasor<0>(phase_cycles(c, rec[0], rec[1], rec[2], rec[3]), T, &gr, &gi);
      visit(k, gr, gi);
    }
  } else {
    // One run at a time: its top (up to) four bins evaluated directly give
    // the backward differences; every bin of the run in this block is then
    // visited from one call site (direct phases for the top bins, the
    // recurrence below them), which keeps the loop body small.  A block
    // that starts inside a run advances the recurrence through the run's
    // bins above it without visiting them.
    const double lin_step = -c.a8 * df;  // linear phase change per bin of the descending walk
    int k = ke - 1;
    while (k >= kb) {
      int L = 0, s = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int sj = k & ~(R.len[j] - 1);
        if (L == 0 && sj >= R.k_min[j]) {
          L = R.len[j];
          s = sj;
        }
      }
      // a bin below the lowest level is a run of one, evaluated directly
      const int top = L == 0 ? k : (s + L - 1 < n_freq - 1 ? s + L - 1 : n_freq - 1);
      if (L == 0) s = k;
      const int nd = top - s + 1 < 4 ? top - s + 1 : 4;
      double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;  // direct phases of bins top, top - 1, ...
      double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0, lin = 0.0;
#pragma nounroll
      for (int j = 0; j < nd; ++j) {
        const double* __restrict__ rc = bins + (int64_t)(top - j) * RS;
        const double nl = phase_nonlinear(c, rc[0], rc[1], rc[2], rc[3]);
        lin = fma(c.a8, rc[0] * rc[1], c.a5);
        const double d1 = nl - n0;
        const double d2 = d1 - n1;
        n3 = d2 - n2;
        n2 = d2;
        n1 = d1;
        n0 = nl;
        const double ph = nl + lin;
        r0 = j == 0 ? ph : r0;
        r1 = j == 1 ? ph : r1;
        r2 = j == 2 ? ph : r2;
        r3 = j == 3 ? ph : r3;
      }
      double p0 = n0 + lin, p1 = n1 + lin_step, p2 = n2;
      const double p3 = n3;
      int kk = top - nd;
      for (; kk > k; --kk) {  // above the walk's first bin: advance only
        p2 += p3;
        p1 += p2;
        p0 += p1;
      }
      const int lo = s > kb ? s : kb;
      for (kk = k; kk >= lo; --kk) {
        const int j = top - kk;
        double ph;
        if (j < nd) {
          ph = j == 0 ? r0 : (j == 1 ? r1 : (j == 2 ? r2 : r3));
        } else {
          p2 += p3;
          p1 += p2;
          p0 += p1;
          ph = p0;
        }
        double gr, gi;
        tm_phasor<1>(ph, T, &gr, &gi);
        visit(kk, gr, gi);
      }
      k = s - 1;
    }
  }
  if (p >= n) return;
  double* __restrict__ out = mom + (p * K * n_blk + b) * 2;
#pragma unroll
  for (int m = 0; m < K; ++m) {
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

template <int ND, int K>
static void launch_tmom_k(gw_ctx* ctx, const double* coef, int64_t ld, int64_t n, int prec, int blk, int n_blk,
                          int tpb, double* mom, hipStream_t st) {
  const int64_t nptile = (n + tpb - 1) / tpb;
  const TrigConsts T = make_trig_consts();
  const PhaseRuns R = make_phase_runs(ctx->geom);
  if (prec == GW_PREC_FP64)
    hipLaunchKernelGGL((k_tmom<ND, 0, K>), dim3((unsigned)(nptile * n_blk)), dim3(tpb), 0, st, coef, ld, n,
                       ctx->bins, ctx->geom.k0, ctx->geom.df, (int)ctx->geom.n_freq, blk, n_blk, T, R, 1.0, 0.0,
                       (const double*)ctx->tm_basis, mom);
  else
    hipLaunchKernelGGL((k_tmom<ND, 1, K>), dim3((unsigned)(nptile * n_blk)), dim3(tpb), 0, st, coef, ld, n,
                       ctx->bins, ctx->geom.k0, ctx->geom.df, (int)ctx->geom.n_freq, blk, n_blk, T, R,
                       ctx->pgain_re, ctx->pgain_im, (const double*)ctx->tm_basis, mom);
}

template <int ND>
static void launch_tmom_nd(gw_ctx* ctx, const double* coef, int64_t ld, int64_t n, int prec, int K, int blk,
                           int n_blk, int tpb, double* mom, hipStream_t st) {
  if (K == 12)
    launch_tmom_k<ND, 12>(ctx, coef, ld, n, prec, blk, n_blk, tpb, mom, st);
  else
    launch_tmom_k<ND, 16>(ctx, coef, ld, n, prec, blk, n_blk, tpb, mom, st);
}

// Grid of the time marginal for the context's window: N, J, P, B.
struct TimeGrid {
  int64_t N;
  double delta;  // the segment's sampling interval; the grid step is delta / R
  int J, R, P, blk, n_blk;
  int L;  // transform length P R
};

static gw_status time_grid(const gw_ctx* ctx, TimeGrid* g) {
  const int64_t top = 2 * (ctx->geom.k0 + ctx->geom.n_freq - 1);
  int64_t N = 1;
  while (N < top) N <<= 1;
  g->N = N;
  g->delta = 1.0 / ((double)N * ctx->geom.df);
  g->J = (int)floor(ctx->tm_window / g->delta + 1e-9);
  g->R = ctx->tm_R;
  // P >= 2 J + 1, and at least 16 / R so that the transform has 16 points
  int P = 2;
  while (P < 2 * g->J + 1 || P * g->R < 16) P <<= 1;
  if (P > kTMaxP) return set_error(GW_ENOTSUP, "time marginal: window %.6g s needs more than %d grid points",
                                   ctx->tm_window, kTMaxP);
  if (N / P < 1) return set_error(GW_ENOTSUP, "time marginal: grid finer than the segment's sampling");
  g->P = P;
  g->blk = (int)(N / P);
  g->n_blk = (int)((ctx->geom.n_freq + g->blk - 1) / g->blk);
  g->L = P * g->R;
  int D1, D2;
  if (!tgrid_plan(g->L, &D1, &D2))
    return set_error(GW_ENOTSUP, "time marginal: %d grid points per sampling interval over +-%.6g s need a "
                                 "%d-point transform (at most 4096)", g->R, ctx->tm_window, g->L);
  return GW_OK;
}

gw_status time_grid_shape(const gw_ctx* ctx, TimeGridShape* out) {
  TimeGrid g;
  const gw_status s = time_grid(ctx, &g);
  if (s != GW_OK) return s;
  out->N = g.N;
  out->delta = g.delta;
  out->J = g.J;
  out->R = g.R;
  out->P = g.P;
  out->blk = g.blk;
  out->n_blk = g.n_blk;
  out->L = g.L;
  out->jmax = g.J * g.R;
  return GW_OK;
}

gw_status loglike_tmarg(gw_ctx* ctx, const double* theta, int64_t n, int prec, double* logl, hipStream_t st) {
  return loglike_tmarg_staged(ctx, theta, n, prec, logl, nullptr, st);
}

gw_status loglike_tmarg_staged(gw_ctx* ctx, const double* theta, int64_t n, int prec, double* logl, double* zout,
                               hipStream_t st) {
  TimeGrid g;
  gw_status s = time_grid(ctx, &g);
  const int K = tgrid_orders(g.L, g.J * g.R);
  if (s == GW_OK) s = tgrid_tables(ctx, g.L, g.J * g.R, K);
  if (s != GW_OK) return s;
  if (ctx->tm_basis_blk != g.blk || ctx->tm_basis_K != K) {
    std::vector<double> h;
    tgrid_basis(g.blk, K, &h);
    if (ctx->tm_basis) (void)hipFree(ctx->tm_basis);
    ctx->tm_basis = nullptr;
    ctx->tm_basis_blk = 0;
    s = check_hip(hipMalloc((void**)&ctx->tm_basis, h.size() * sizeof(double)), "time-grid basis");
    if (s == GW_OK)
      s = check_hip(hipMemcpy(ctx->tm_basis, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice), "basis");
    if (s != GW_OK) return s;
    ctx->tm_basis_blk = g.blk;
    ctx->tm_basis_K = K;
  }
  const int64_t chunk = tgrid_chunk_rows(n, g.n_blk, K);
  const int nt = 2 * g.J * g.R + 1;
  // workspace: the moments of a row chunk, then the order groups' partial
  // grids of a small launch
  const int64_t zp = tgrid_zpart_elems(n, chunk, K, nt);
  s = ensure_buffer(&ctx->coef, &ctx->coef_cap, (int64_t)C_NCOEF * n, "coefficient workspace");
  if (s == GW_OK)
    s = ensure_buffer(&ctx->tm_mom, &ctx->tm_mom_cap, chunk * K * g.n_blk * 2 + 2 * zp, "time moments");
  if (s != GW_OK || !theta) return s;  // theta NULL: reserve only
  s = launch_prologue(ctx, theta, n, GW_MARG_PHASE_TIME, ctx->coef, n, st);
  if (s != GW_OK) return s;
  for (int64_t r0 = 0; r0 < n && s == GW_OK; r0 += chunk) {
    const int64_t cn = n - r0 < chunk ? n - r0 : chunk;
    const int tpb = cn >= 2048 ? 256 : 64;
    const int slot = prof_begin(ctx, st, 1);
    switch (ctx->n_det) {
      case 1: launch_tmom_nd<1>(ctx, ctx->coef + r0, n, cn, prec, K, g.blk, g.n_blk, tpb, ctx->tm_mom, st); break;
      case 2: launch_tmom_nd<2>(ctx, ctx->coef + r0, n, cn, prec, K, g.blk, g.n_blk, tpb, ctx->tm_mom, st); break;
      case 3: launch_tmom_nd<3>(ctx, ctx->coef + r0, n, cn, prec, K, g.blk, g.n_blk, tpb, ctx->tm_mom, st); break;
      case 4: launch_tmom_nd<4>(ctx, ctx->coef + r0, n, cn, prec, K, g.blk, g.n_blk, tpb, ctx->tm_mom, st); break;
      default: return set_error(GW_ENOTSUP, "n_det %d not supported", ctx->n_det);
    }
    prof_end(ctx, slot, st);
    s = check_hip(hipGetLastError(), "time moments launch");
    if (s != GW_OK) return s;
    TGridArgs a{};
    a.mom = ctx->tm_mom;
    a.mom_rs = (int64_t)K * g.n_blk;  // k_tmom writes one row's moments contiguously
    a.mom_es = 1;
    a.n = cn;
    a.n_blk = g.n_blk;
    a.L = g.L;
    a.jmax = g.J * g.R;
    a.K = K;
    a.coef = ctx->coef + r0;
    a.ld = n;
    a.logl = logl + r0;
    a.zout = zout ? zout + r0 * nt * 3 : nullptr;
    a.f0_num = (double)(2 * ctx->geom.k0 + g.blk - 1);
    a.f0_den = (double)(2 * g.N) * (double)g.R;
    a.zpart = zp > 0 ? ctx->tm_mom + chunk * K * g.n_blk * 2 : nullptr;
    const int gslot = prof_begin(ctx, st, 2);
    s = launch_tgrid(ctx, a, st);
    prof_end(ctx, gslot, st);
  }
  return s;
}

gw_status tmarg_reserve(gw_ctx* ctx, int64_t n, int like) {
  return like == GW_HET ? loglike_het_tmarg_staged(ctx, nullptr, n, GW_PREC_FP64, nullptr, nullptr, 0)
                        : loglike_tmarg_staged(ctx, nullptr, n, GW_PREC_FP64, nullptr, nullptr, 0);
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
  else ++ctx->gen;
  return s;
}

extern "C" gw_status gw_set_time_oversample(gw_ctx* ctx, int32_t factor) {
  if (!ctx) return gw::set_error(GW_EINVAL, "gw_set_time_oversample: ctx is NULL");
  if (factor != 1 && factor != 2 && factor != 4 && factor != 8 && factor != 16)
    return gw::set_error(GW_EINVAL, "gw_set_time_oversample: factor must be 1, 2, 4, 8 or 16");
  ctx->tm_R = factor;
  ++ctx->gen;
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
