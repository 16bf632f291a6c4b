// Post-hoc reconstruction of the marginalised distance and phase (appendix on
// grid marginalisations).  For each posterior sample the likelihood kernels
// stage the sample's overlap Z and norm <h|h> (at d_L = 1 Mpc for the distance
// marginal, phi_c = 0); one wave per sample then draws
//   * d_j from exp(ln w_j - <h|h>_1 / (2 d_j^2) + ln I0(|Z_1| / d_j)) on the
//     distance grid (the terms of the distance-marginal log-sum-exp), and
//   * phi_c given d_j from exp(kappa cos(phi + arg Z)), kappa = |Z| / d_j, on
//     the uniform phase grid phi_m = 2 pi m / N_phi (the dense-grid form of
//     the phase marginal of Sec. III.A; the template carries exp(+i phi_c)),
// each by inverting the cumulative grid weights: the first index whose
// cumulative weight exceeds u times the total.
#include "gw_ctx.h"

namespace gw {

// Inverse-CDF draw over a grid of len points, by one wave.  Lane l owns the
// contiguous points [l s, (l + 1) s), s = ceil(len / 64); weights are
// exp(logw(j) - shift) with shift >= max logw.  The lane sums are scanned over
// the lanes in lane order; the lane whose [exclusive, inclusive) range holds
// u * total rescans its points.  Every lane returns the drawn index.
template <class F>
__device__ inline int wave_draw(const F& logw, int len, double shift, double u, int lane) {
  const int per = (len + 63) / 64;
  const int lo = lane * per < len ? lane * per : len;
  const int hi = lo + per < len ? lo + per : len;
  double s = 0.0;
  for (int j = lo; j < hi; ++j) s += exp(logw(j) - shift);
  double incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  double excl = __shfl_up(incl, 1, 64);
  if (lane == 0) excl = 0.0;
  const double total = __shfl(incl, 63, 64);
  const double t = u * total;
  const bool claim = s > 0.0 && excl <= t && t < incl;
  int pick = -1;
  if (claim) {
    double c = excl;
    for (int j = lo; j < hi; ++j) {
      const double w = exp(logw(j) - shift);
      c += w;
      if (w > 0.0) pick = j;  // the last positive point unless the crossing comes first
      if (c > t && w > 0.0) break;
    }
  }
  const unsigned long long m = __ballot(claim);
  if (m) return __shfl(pick, __ffsll((long long)m) - 1, 64);
  // u * total rounded up to the total: the last point with positive weight
  int last = -1;
  for (int j = lo; j < hi; ++j)
    if (exp(logw(j) - shift) > 0.0) last = j;
  const unsigned long long h = __ballot(last >= 0);
  if (!h) return -1;
  return __shfl(last, 63 - __clzll((long long)h), 64);
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Full band: (Re Z, Im Z, <h|h>) per row from the per-detector sums z_i and
// the prologue's prefactors A P_i, in the epilogue's order.
__global__ void __launch_bounds__(256) k_recon_stage(const double* __restrict__ zrow, int nd,
                                                     const double* __restrict__ coef, int64_t ld, int64_t n,
                                                     double* __restrict__ zc3) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double Zr = 0.0, Zi = 0.0;
  for (int i = 0; i < nd; ++i) {
    const double zr = zrow[p * 2 * nd + 2 * i], zi = zrow[p * 2 * nd + 2 * i + 1];
    const double ar = coef[(C_APRE + i) * ld + p];
    const double ai = coef[(C_APIM + i) * ld + p];
    Zr += ar * zr - ai * zi;
    Zi += ar * zi + ai * zr;
  }
  const bool valid = coef[C_VALID * ld + p] != 0.0;
  zc3[p] = valid ? Zr : NAN;
  zc3[n + p] = Zi;
  zc3[2 * n + p] = coef[C_HH * ld + p];
}

// One wave per sample: out[p] = (d_L, phi_c), idx[p] = (j, m) or (-1, m) when
// d_L is the sample's own (phase marginal); NaN and -1 for unphysical rows.
__global__ void __launch_bounds__(256) k_recon(const double* __restrict__ zc3, int64_t n,
                                               const double* __restrict__ theta, const double* __restrict__ tab,
                                               int n_dist, int marg, int n_phase,
                                               const double* __restrict__ uni, double* __restrict__ out,
                                               int32_t* __restrict__ idx) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (p >= n) return;  // wave-uniform
  const double zr = zc3[p], zi = zc3[n + p], hh = zc3[2 * n + p];
  auto invalid = [&]() {
    if (lane == 0) {
      out[2 * p] = NAN;
      out[2 * p + 1] = NAN;
      if (idx) {
        idx[2 * p] = -1;
        idx[2 * p + 1] = -1;
      }
    }
  };
  if (isnan(zr)) return invalid();
  double d, zpr, zpi;
  int j = -1;
  if (marg == GW_MARG_PHASE_DIST) {
    const double za = sqrt(zr * zr + zi * zi);
    auto lw = [&](int q) {
      const double* r = tab + 4 * q;
      return fma(-hh, r[2], r[3]) + log_i0(za * r[1]);
    };
    double mx = -INFINITY;
    for (int q = lane; q < n_dist; q += 64) mx = fmax(mx, lw(q));
    mx = wave_max(mx);
    j = wave_draw(lw, n_dist, mx, uni[2 * p], lane);
    if (j < 0) return invalid();  // no finite weight (non-finite overlap)
    d = tab[4 * j];
    zpr = zr * tab[4 * j + 1];
    zpi = zi * tab[4 * j + 1];
  } else {
    d = theta[p * 13 + 6];
    zpr = zr;
    zpi = zi;
  }
  // kappa cos(phi_m + arg Z) = Re Z cos(phi_m) - Im Z sin(phi_m), at most kappa
  const double kappa = sqrt(zpr * zpr + zpi * zpi);
  const double dphi = kTwoPi / (double)n_phase;
  auto pw = [&](int q) {
    double sn, cs;
    sincos(dphi * (double)q, &sn, &cs);
    return zpr * cs - zpi * sn;
  };
  const int m = wave_draw(pw, n_phase, kappa, uni[2 * p + 1], lane);
  if (m < 0) return invalid();
  if (lane == 0) {
    out[2 * p] = d;
    out[2 * p + 1] = kTwoPi * (double)m / (double)n_phase;
    if (idx) {
      idx[2 * p] = j;
      idx[2 * p + 1] = m;
    }
  }
}

// Stage (Re Z, Im Z, <h|h>) of n rows in ctx->recon [3][n] (Re Z NaN for
// unphysical rows) and their marginal log L in logl (or in the work space).
gw_status stage_overlaps(gw_ctx* ctx, const double* theta, int64_t n, int like, int marg, int prec, double* logl,
                         hipStream_t st) {
  const int nd = ctx->n_det;
  gw_status s = ensure_buffer(&ctx->recon, &ctx->recon_cap, (int64_t)(3 + 2 * nd + 1) * n, "reconstruction workspace");
  if (s != GW_OK) return s;
  double* zc3 = ctx->recon;
  double* zrow = zc3 + 3 * n;
  double* ll = logl ? logl : zrow + 2 * nd * n;
  if (like == GW_HET) return loglike_het_staged(ctx, theta, n, marg, prec, ll, zc3, st);
  int tpb, nch;
  full_launch_shape(ctx, n, &tpb, &nch);
  s = ensure_buffer(&ctx->coef, &ctx->coef_cap, (int64_t)C_NCOEF * n, "coefficient workspace");
  if (s == GW_OK) s = ensure_buffer(&ctx->partial, &ctx->partial_cap, (int64_t)nch * 2 * nd * n, "partials");
  if (s == GW_OK) s = ensure_buffer(&ctx->zbuf, &ctx->zbuf_cap, 2 * n, "marginal workspace");
  if (s == GW_OK) s = launch_prologue(ctx, theta, n, marg, ctx->coef, n, st);
  if (s == GW_OK) s = launch_full(ctx, ctx->coef, n, n, prec, tpb, nch, ctx->partial, st);
  if (s == GW_OK)
    s = launch_epilogue_cached(ctx, ctx->partial, nch, ctx->coef, n, n, marg, prec, ll, nullptr, nullptr, zrow, st);
  if (s != GW_OK) return s;
  hipLaunchKernelGGL(k_recon_stage, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, zrow, nd, ctx->coef, n, n,
                     zc3);
  return check_hip(hipGetLastError(), "reconstruction staging launch");
}

// Phase+time marginal: one wave per sample draws t_j from
// exp(-<h|h>(t_j)/2 + ln I0(|Z(t_j)|)) on the staged grid values
// zt [n][nt][3], then phi_c from exp(|Z(t_j)| cos(phi + arg Z(t_j))).
// out[p] = (t_j, phi_c) with t_j = (j - J) delta; idx[p] = (j, m).
__global__ void __launch_bounds__(256) k_recon_time(const double* __restrict__ zt, int64_t n, int nt, int J,
                                                    double delta, int n_phase,
                                                    const double* __restrict__ uni, double* __restrict__ out,
                                                    int32_t* __restrict__ idx) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (p >= n) return;  // wave-uniform
  const double* z = zt + p * nt * 3;
  auto invalid = [&]() {
    if (lane == 0) {
      out[2 * p] = NAN;
      out[2 * p + 1] = NAN;
      if (idx) {
        idx[2 * p] = -1;
        idx[2 * p + 1] = -1;
      }
    }
  };
  if (isnan(z[0])) return invalid();
  auto lw = [&](int q) {
    const double* r = z + 3 * q;
    return -0.5 * r[2] + log_i0(sqrt(r[0] * r[0] + r[1] * r[1]));
  };
  double mx = -INFINITY;
  for (int q = lane; q < nt; q += 64) mx = fmax(mx, lw(q));
  mx = wave_max(mx);
  const int j = wave_draw(lw, nt, mx, uni[2 * p], lane);
  if (j < 0) return invalid();
  const double zpr = z[3 * j], zpi = z[3 * j + 1];
  const double kappa = sqrt(zpr * zpr + zpi * zpi);
  const double dphi = kTwoPi / (double)n_phase;
  auto pw = [&](int q) {
    double sn, cs;
    sincos(dphi * (double)q, &sn, &cs);
    return zpr * cs - zpi * sn;
  };
  const int m = wave_draw(pw, n_phase, kappa, uni[2 * p + 1], lane);
  if (m < 0) return invalid();
  if (lane == 0) {
    out[2 * p] = (double)(j - J) * delta;
    out[2 * p + 1] = kTwoPi * (double)m / (double)n_phase;
    if (idx) {
      idx[2 * p] = j;
      idx[2 * p + 1] = m;
    }
  }
}

}  // namespace gw

using namespace gw;

extern "C" {

gw_status gw_reconstruct(gw_ctx* ctx, const double* theta, int64_t n, int32_t like, int32_t marg, int32_t prec,
                         const double* uniforms, int32_t n_phase, double* out, int32_t* idx, double* logl,
                         void* stream) {
  if (!ctx) return set_error(GW_EINVAL, "gw_reconstruct: ctx is NULL");
  if (n < 0) return set_error(GW_EINVAL, "gw_reconstruct: n < 0");
  if (n > 0 && (!theta || !uniforms || !out)) return set_error(GW_EINVAL, "gw_reconstruct: null pointer");
  if (like != GW_FULL && like != GW_HET) return set_error(GW_EINVAL, "gw_reconstruct: bad like=%d", like);
  if (marg != GW_MARG_PHASE && marg != GW_MARG_PHASE_DIST && marg != GW_MARG_PHASE_TIME)
    return set_error(GW_ENOTSUP, "gw_reconstruct: marg must be GW_MARG_PHASE, GW_MARG_PHASE_DIST or GW_MARG_PHASE_TIME");
  if (prec != GW_PREC_FP64 && prec != GW_PREC_MIXED) return set_error(GW_EINVAL, "gw_reconstruct: bad prec=%d", prec);
  if (n_phase < 1 || n_phase > (1 << 20)) return set_error(GW_EINVAL, "gw_reconstruct: n_phase 1 .. 2^20");
  if (marg == GW_MARG_PHASE_DIST && ctx->n_dist <= 0)
    return set_error(GW_ESTATE, "gw_reconstruct: distance marginal needs a distance grid");
  if (like == GW_HET && !ctx->het) return set_error(GW_ESTATE, "gw_reconstruct: heterodyne_setup has not been called");
  if (n == 0) return GW_OK;
  hipStream_t st = (hipStream_t)stream;
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  if (marg == GW_MARG_PHASE_TIME) {
    double delta;
    int32_t nt;
    s = gw_time_grid_info(ctx, &delta, &nt, nullptr, nullptr);
    if (s == GW_OK)
      s = ensure_buffer(&ctx->recon, &ctx->recon_cap, (int64_t)nt * 3 * n + n, "reconstruction workspace");
    if (s != GW_OK) return s;
    double* zt = ctx->recon;
    double* ll = logl ? logl : zt + (int64_t)nt * 3 * n;
    s = like == GW_HET ? loglike_het_tmarg_staged(ctx, theta, n, prec, ll, zt, st)
                       : loglike_tmarg_staged(ctx, theta, n, prec, ll, zt, st);
    if (s != GW_OK) return s;
    hipLaunchKernelGGL(k_recon_time, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, zt, n, nt, (nt - 1) / 2, delta,
                       n_phase, uniforms, out, idx);
    return check_hip(hipGetLastError(), "time reconstruction launch");
  }
  s = stage_overlaps(ctx, theta, n, like, marg, prec, logl, st);
  if (s != GW_OK) return s;
  double* zc3 = ctx->recon;
  hipLaunchKernelGGL(k_recon, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, zc3, n, theta, ctx->dist_tab,
                     ctx->n_dist, marg, n_phase, uniforms, out, idx);
  return check_hip(hipGetLastError(), "reconstruction launch");
}

}  // extern "C"
