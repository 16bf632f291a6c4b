// Maximum-likelihood search for the heterodyne fiducial (the GW170817
// section takes the reference parameters of the relative binning from a
// maximum-likelihood optimisation over priors narrowed to the event).  The
// optimiser is differential evolution, DE/rand/1/bin (Storn & Price 1997),
// over a box of the sampler's unit cube; a generation is one trial kernel,
// the prior transform and one batched full-band likelihood call, and one
// selection kernel.
#include <cmath>
#include <vector>

#include "gw_ctx.h"
#include "gw_rng.h"

namespace gw {

constexpr int kDeDim = 11;

struct DeBox {
  double lo[kDeDim], hi[kDeDim];
};

// The k-th (from 0) index not among the ascending exclusions e[0..n).
__device__ inline int64_t kth_excluding(int64_t k, const int64_t* e, int n) {
  for (int a = 0; a < n; ++a)
    if (k >= e[a]) ++k;
  return k;
}

__device__ inline void sort_small(int64_t* e, int n) {
  for (int a = 1; a < n; ++a)
    for (int b = a; b > 0 && e[b - 1] > e[b]; --b) {
      const int64_t t = e[b];
      e[b] = e[b - 1];
      e[b - 1] = t;
    }
}

// Trial of member i in generation gen.  Uniform j is Philox word j % 4 of
// counter (gen, i, j / 4, 0) under key (seed, 2): u_0..u_2 choose three
// distinct partners other than i (each the k-th remaining index, k =
// floor(u (P - 1 - m)) after m exclusions), u_3 the coordinate always
// crossed, u_(4+j) < CR crosses coordinate j.  Mutant x_r1 + F (x_r2 - x_r3)
// without fused multiply-add; coordinates outside the box are mirrored at
// its walls and clipped.
__global__ void __launch_bounds__(256) k_de_trial(const double* __restrict__ x, int64_t pop, DeBox box, uint64_t gen,
                                                  uint64_t seed, double f_scale, double cr, double* __restrict__ t) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pop) return;
  double u[16];
  for (int b = 0; b < 4; ++b) {
    uint64_t c[4] = {gen, (uint64_t)i, (uint64_t)b, 0ull};
    philox4x64(c, seed, 2ull);
    for (int w = 0; w < 4; ++w) u[4 * b + w] = philox_unit(c[w]);
  }
  int64_t ex[3] = {i, 0, 0};
  const int64_t r1 = kth_excluding((int64_t)floor(u[0] * (double)(pop - 1)), ex, 1);
  ex[1] = r1;
  sort_small(ex, 2);
  const int64_t r2 = kth_excluding((int64_t)floor(u[1] * (double)(pop - 2)), ex, 2);
  ex[2] = r2;
  sort_small(ex, 3);
  const int64_t r3 = kth_excluding((int64_t)floor(u[2] * (double)(pop - 3)), ex, 3);
  const int jrand = (int)floor(u[3] * (double)kDeDim);
  for (int j = 0; j < kDeDim; ++j) {
    double v = x[i * kDeDim + j];
    if (j == jrand || u[4 + j] < cr) {
      const double d = x[r2 * kDeDim + j] - x[r3 * kDeDim + j];
      const double s = f_scale * d;
      v = x[r1 * kDeDim + j] + s;
      const double lo = box.lo[j], hi = box.hi[j];
      if (v < lo) v = lo + (lo - v);
      else if (v > hi) v = hi - (v - hi);
      v = fmin(hi, fmax(lo, v));
    }
    t[i * kDeDim + j] = v;
  }
}

// Greedy selection: the trial replaces member i when its log L is not NaN and
// at least the member's (or the member's is NaN).
__global__ void __launch_bounds__(256) k_de_select(double* __restrict__ x, double* __restrict__ fx,
                                                   const double* __restrict__ t, const double* __restrict__ ft,
                                                   int64_t pop) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pop) return;
  const double a = ft[i], b = fx[i];
  if (isnan(a) || !(a >= b || isnan(b))) return;
  for (int j = 0; j < kDeDim; ++j) x[i * kDeDim + j] = t[i * kDeDim + j];
  fx[i] = a;
}

}  // namespace gw

using namespace gw;

extern "C" {

gw_status gw_fiducial_search(gw_ctx* ctx, const gw_fiducial_args* a, double* x, double* fx, double* theta_best,
                             void* stream) {
  if (!ctx || !a) return set_error(GW_EINVAL, "gw_fiducial_search: null argument");
  if (!x || !fx || !theta_best) return set_error(GW_EINVAL, "gw_fiducial_search: null pointer");
  const int64_t pop = a->pop;
  if (pop < 4 || pop > (1 << 22)) return set_error(GW_EINVAL, "gw_fiducial_search: pop 4 .. 2^22");
  if (a->generations < 0) return set_error(GW_EINVAL, "gw_fiducial_search: generations < 0");
  if (!(a->f_scale > 0.0 && a->f_scale <= 2.0)) return set_error(GW_EINVAL, "gw_fiducial_search: F in (0, 2]");
  if (!(a->cr >= 0.0 && a->cr <= 1.0)) return set_error(GW_EINVAL, "gw_fiducial_search: CR in [0, 1]");
  if (a->prec != GW_PREC_FP64 && a->prec != GW_PREC_MIXED)
    return set_error(GW_EINVAL, "gw_fiducial_search: bad prec=%d", a->prec);
  if (ctx->n_dist <= 0) return set_error(GW_ESTATE, "gw_fiducial_search: needs a distance grid");
  DeBox box;
  for (int j = 0; j < kDeDim; ++j) {
    box.lo[j] = a->lo ? a->lo[j] : 0.0;
    box.hi[j] = a->hi ? a->hi[j] : 1.0;
    if (!(box.lo[j] >= 0.0 && box.lo[j] <= box.hi[j] && box.hi[j] <= 1.0))
      return set_error(GW_EINVAL, "gw_fiducial_search: coordinate %d: need 0 <= lo <= hi <= 1", j);
  }
  hipStream_t st = (hipStream_t)stream;
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  // work space: trials [pop][11], parameter vectors [pop][13], trial log L [pop]
  double* ws = nullptr;
  s = check_hip(hipMalloc((void**)&ws, (size_t)pop * (kDeDim + 13 + 1) * sizeof(double)), "fiducial workspace");
  if (s != GW_OK) return s;
  double* t = ws;
  double* th = t + pop * kDeDim;
  double* ft = th + pop * 13;
  const int marg = GW_MARG_PHASE_DIST;
  const unsigned grid = (unsigned)((pop + 255) / 256);
  s = gw_prior_transform_marg(ctx, x, pop, marg, th, stream);
  if (s == GW_OK) s = loglike_batch(ctx, th, pop, GW_FULL, marg, a->prec, fx, stream);
  for (int g = 0; g < a->generations && s == GW_OK; ++g) {
    hipLaunchKernelGGL(k_de_trial, dim3(grid), dim3(256), 0, st, x, pop, box, (uint64_t)g, a->seed, a->f_scale,
                       a->cr, t);
    s = check_hip(hipGetLastError(), "trial launch");
    if (s == GW_OK) s = gw_prior_transform_marg(ctx, t, pop, marg, th, stream);
    if (s == GW_OK) s = loglike_batch(ctx, th, pop, GW_FULL, marg, a->prec, ft, stream);
    if (s == GW_OK) {
      hipLaunchKernelGGL(k_de_select, dim3(grid), dim3(256), 0, st, x, fx, t, ft, pop);
      s = check_hip(hipGetLastError(), "selection launch");
    }
  }
  // best member, then its (d_L, phi_c) at the peak of the plain likelihood:
  // Re(Z_1 e^{i phi}) / d - <h|h>_1 / (2 d^2) is largest at phi = -arg Z_1,
  // d = <h|h>_1 / |Z_1|
  std::vector<double> hf((size_t)pop);
  if (s == GW_OK) s = check_hip(hipMemcpyAsync(hf.data(), fx, pop * sizeof(double), hipMemcpyDeviceToHost, st), "copy");
  if (s == GW_OK) s = check_hip(hipStreamSynchronize(st), "sync");
  int64_t best = -1;
  if (s == GW_OK) {
    for (int64_t i = 0; i < pop; ++i)
      if (!std::isnan(hf[i]) && hf[i] > -INFINITY && (best < 0 || hf[i] > hf[best])) best = i;
    if (best < 0) s = set_error(GW_EDEVICE, "gw_fiducial_search: no member has a finite likelihood");
  }
  if (s == GW_OK) s = gw_prior_transform_marg(ctx, x + best * kDeDim, 1, marg, th, stream);
  if (s == GW_OK) s = stage_overlaps(ctx, th, 1, GW_FULL, marg, GW_PREC_FP64, ft, st);
  double zc[3] = {0, 0, 0};
  if (s == GW_OK)
    s = check_hip(hipMemcpyAsync(theta_best, th, 13 * sizeof(double), hipMemcpyDeviceToHost, st), "copy");
  if (s == GW_OK) {
    for (int q = 0; q < 3 && s == GW_OK; ++q)
      s = check_hip(hipMemcpyAsync(&zc[q], ctx->recon + q, sizeof(double), hipMemcpyDeviceToHost, st), "copy");
  }
  if (s == GW_OK) s = check_hip(hipStreamSynchronize(st), "sync");
  (void)hipFree(ws);
  if (s != GW_OK) return s;
  const double za = std::sqrt(zc[0] * zc[0] + zc[1] * zc[1]);
  if (!(za > 0.0)) return set_error(GW_EDEVICE, "gw_fiducial_search: the best point has no overlap with the data");
  double phi = -std::atan2(zc[1], zc[0]);
  if (phi < 0.0) phi += kTwoPi;
  theta_best[6] = zc[2] / za;
  theta_best[11] = phi;
  return GW_OK;
}

}  // extern "C"
