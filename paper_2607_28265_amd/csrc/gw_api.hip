// C ABI of libgwswig: context lifetime, error reporting and the batched
// full-band likelihood entry points.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gw_ctx.h"

namespace {
thread_local char g_err[512] = "";
}

namespace gw {

gw_status set_error(gw_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

gw_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return GW_OK;
  if (e == hipErrorOutOfMemory) return set_error(GW_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return set_error(GW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Optional fault injection for error-path tests: GW_FAULT=alloc makes every
// workspace allocation fail.
static bool fault_alloc() {
  const char* f = getenv("GW_FAULT");
  return f && strcmp(f, "alloc") == 0;
}

gw_status ensure_buffer(double** buf, int64_t* cap, int64_t need, const char* what) {
  if (need <= *cap) return GW_OK;
  if (fault_alloc()) return set_error(GW_ENOMEM, "%s: injected allocation failure", what);
  if (*buf) {
    hipError_t e = hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    if (e != hipSuccess) return check_hip(e, what);
  }
  double* p = nullptr;
  hipError_t e = hipMalloc((void**)&p, (size_t)need * sizeof(double));
  if (e != hipSuccess) return check_hip(e, what);
  *buf = p;
  *cap = need;
  return GW_OK;
}

// Neumaier-compensated sum, used for the host-side constants.
struct CompSum {
  double s = 0.0, c = 0.0;
  void add(double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

constexpr int kProfSlots = 4096;

int prof_begin(gw_ctx* ctx, hipStream_t st, int which) {
  if (ctx->prof != which || ctx->prof_used >= kProfSlots) return -1;
  if (ctx->prof_ev.empty()) {
    ctx->prof_ev.resize(2 * kProfSlots, nullptr);
  }
  const int slot = ctx->prof_used;
  for (int j = 0; j < 2; ++j)
    if (!ctx->prof_ev[2 * slot + j] && hipEventCreate(&ctx->prof_ev[2 * slot + j]) != hipSuccess) return -1;
  if (hipEventRecord(ctx->prof_ev[2 * slot], st) != hipSuccess) return -1;
  return slot;
}

void prof_end(gw_ctx* ctx, int slot, hipStream_t st) {
  if (slot < 0) return;
  if (hipEventRecord(ctx->prof_ev[2 * slot + 1], st) == hipSuccess) ctx->prof_used = slot + 1;
}

}  // namespace gw

using namespace gw;

namespace gw {
gw_status full_reserve(gw_ctx* ctx, int64_t n) {
  int tpb, nch;
  full_launch_shape(ctx, n, &tpb, &nch);
  gw_status s = ensure_buffer(&ctx->coef, &ctx->coef_cap, (int64_t)C_NCOEF * n, "coefficient workspace");
  if (s == GW_OK) s = ensure_buffer(&ctx->partial, &ctx->partial_cap, (int64_t)nch * 2 * ctx->n_det * n, "partials");
  if (s == GW_OK) s = ensure_buffer(&ctx->zbuf, &ctx->zbuf_cap, 2 * n, "marginal workspace");
  return s;
}
}  // namespace gw

extern "C" {

const char* gw_last_error(void) { return g_err; }

const char* gw_version(void) { return "gwswig 0.1 (gfx950)"; }

gw_status gw_ctx_create(const gw_problem* pr, int32_t device, gw_ctx** out) {
  if (!out) return set_error(GW_EINVAL, "gw_ctx_create: out is NULL");
  *out = nullptr;
  if (!pr) return set_error(GW_EINVAL, "gw_ctx_create: problem is NULL");
  if (pr->n_det < 1 || pr->n_det > GW_MAX_DET)
    return set_error(GW_EINVAL, "gw_ctx_create: n_det=%d outside 1..%d", pr->n_det, GW_MAX_DET);
  if (pr->n_freq < 1 || pr->n_freq > (1 << 30))
    return set_error(GW_EINVAL, "gw_ctx_create: n_freq must be in 1 .. 2^30");
  if (pr->k0 < 1) return set_error(GW_EINVAL, "gw_ctx_create: k0 must be >= 1 (f > 0)");
  if (!(pr->df > 0.0) || !isfinite(pr->df)) return set_error(GW_EINVAL, "gw_ctx_create: df must be > 0");
  if (!pr->data_re || !pr->data_im || !pr->psd || !pr->det_tensor || !pr->det_pos)
    return set_error(GW_EINVAL, "gw_ctx_create: null data, psd or detector pointer");
  if (pr->n_dist < 0) return set_error(GW_EINVAL, "gw_ctx_create: n_dist < 0");
  if (pr->n_dist > 0 && (!pr->dist_grid || !pr->dist_logw))
    return set_error(GW_EINVAL, "gw_ctx_create: null distance grid");
  const int nd = pr->n_det;
  const int64_t nf = pr->n_freq;
  for (int64_t j = 0; j < (int64_t)nd * nf; ++j) {
    if (!(pr->psd[j] > 0.0) || !isfinite(pr->psd[j]))
      return set_error(GW_EINVAL, "gw_ctx_create: PSD must be finite and > 0 (index %lld)", (long long)j);
    if (!isfinite(pr->data_re[j]) || !isfinite(pr->data_im[j]))
      return set_error(GW_EINVAL, "gw_ctx_create: data must be finite (index %lld)", (long long)j);
  }
  for (int j = 0; j < pr->n_dist; ++j)
    if (!(pr->dist_grid[j] > 0.0) || !isfinite(pr->dist_logw[j]))
      return set_error(GW_EINVAL, "gw_ctx_create: distance grid must be > 0 with finite weights");

  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) return set_error(GW_EDEVICE, "gw_ctx_create: no HIP device available");
  if (device < 0 || device >= ndev) return set_error(GW_EINVAL, "gw_ctx_create: device %d out of range", device);
  gw_status st = check_hip(hipSetDevice(device), "hipSetDevice");
  if (st == GW_OK) st = noalloc_init(device);  // this device's allocation-free workspace address
  if (st != GW_OK) return st;

  gw_ctx* ctx = new (std::nothrow) gw_ctx();
  if (!ctx) return set_error(GW_ENOMEM, "gw_ctx_create: host allocation");
  ctx->device = device;
  ctx->n_det = nd;
  Geom& g = ctx->geom;
  memset(&g, 0, sizeof(g));
  g.n_det = nd;
  g.k0 = pr->k0;
  g.n_freq = nf;
  g.df = pr->df;
  g.gmst = pr->gmst;
  for (int i = 0; i < nd; ++i) {
    for (int j = 0; j < 9; ++j) g.tensor[i][j] = pr->det_tensor[i * 9 + j];
    for (int j = 0; j < 3; ++j) g.pos[i][j] = pr->det_pos[i * 3 + j];
  }

  // Per-bin records and the closed-form constants.
  const int rs = 4 + 2 * nd;
  ctx->rec_stride = rs;
  std::vector<double> rec((size_t)nf * rs);
  std::vector<CompSum> hw(nd), ddi(nd);
  for (int64_t k = 0; k < nf; ++k) {
    const double f = (double)(pr->k0 + k) * pr->df;
    const double x = cbrt(f);
    double* r = &rec[(size_t)k * rs];
    r[0] = x;
    r[1] = x * x;
    r[2] = pow(f, -5.0 / 3.0);
    r[3] = log(f);
    const double f76 = pow(f, -7.0 / 6.0);
    const double f73 = pow(f, -7.0 / 3.0);
    for (int i = 0; i < nd; ++i) {
      const int64_t j = (int64_t)i * nf + k;
      const double w = 4.0 * pr->df / pr->psd[j];
      r[4 + 2 * i] = w * f76 * pr->data_re[j];
      r[5 + 2 * i] = -w * f76 * pr->data_im[j];
      hw[i].add(w * f73);
      ddi[i].add(w * (pr->data_re[j] * pr->data_re[j] + pr->data_im[j] * pr->data_im[j]));
    }
  }
  CompSum dd;
  for (int i = 0; i < nd; ++i) {
    g.hhw[i] = hw[i].value();
    dd.add(ddi[i].value());
  }
  ctx->dd = dd.value();
  ctx->h_data_re.assign(pr->data_re, pr->data_re + (size_t)nd * nf);
  ctx->h_data_im.assign(pr->data_im, pr->data_im + (size_t)nd * nf);
  ctx->h_psd.assign(pr->psd, pr->psd + (size_t)nd * nf);

  st = check_hip(hipMalloc((void**)&ctx->bins, rec.size() * sizeof(double)), "bins alloc");
  if (st == GW_OK)
    st = check_hip(hipMemcpy(ctx->bins, rec.data(), rec.size() * sizeof(double), hipMemcpyHostToDevice), "bins copy");
  if (st == GW_OK && pr->n_dist > 0) {
    ctx->n_dist = pr->n_dist;
    ctx->h_dist_grid.assign(pr->dist_grid, pr->dist_grid + pr->n_dist);
    ctx->h_dist_logw.assign(pr->dist_logw, pr->dist_logw + pr->n_dist);
    std::vector<double> tab(4 * (size_t)pr->n_dist);
    for (int j = 0; j < pr->n_dist; ++j) {
      const double d = pr->dist_grid[j];
      tab[4 * j] = d;
      tab[4 * j + 1] = 1.0 / d;
      tab[4 * j + 2] = 0.5 / (d * d);
      tab[4 * j + 3] = pr->dist_logw[j];
      ctx->dist_r1max = fmax(ctx->dist_r1max, 1.0 / d);
    }
    st = check_hip(hipMalloc((void**)&ctx->dist_tab, tab.size() * sizeof(double)), "dist alloc");
    if (st == GW_OK)
      st = check_hip(hipMemcpy(ctx->dist_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice),
                     "dist copy");
  }
  if (st == GW_OK) {
    LogI0Consts c = make_log_i0_consts();
    c.r1max = ctx->dist_r1max;
    for (double dj : ctx->h_dist_grid) c.dmax = fmax(c.dmax, dj);
    st = check_hip(hipMalloc((void**)&ctx->i0c, sizeof(LogI0Consts)), "ln I0 table alloc");
    if (st == GW_OK) st = check_hip(hipMemcpy(ctx->i0c, &c, sizeof(c), hipMemcpyHostToDevice), "ln I0 table copy");
  }
  if (st == GW_OK) st = build_moment_table(ctx, rec, pr->det_pos);
  if (st == GW_OK) st = wmom_init(ctx);
  if (st == GW_OK) st = calibrate_phasor(ctx);
  if (st != GW_OK) {
    gw_ctx_destroy(ctx);
    return st;
  }
  *out = ctx;
  return GW_OK;
}

gw_status gw_ctx_destroy(gw_ctx* ctx) {
  if (!ctx) return GW_OK;
  (void)hipSetDevice(ctx->device);
  het_free(ctx);
  graphs_free(ctx);
  slice_free(ctx);
  for (hipEvent_t e : ctx->prof_ev)
    if (e) (void)hipEventDestroy(e);
  double* bufs[] = {ctx->bins,   ctx->dist_tab, ctx->coef,   ctx->partial, ctx->zbuf,
                    ctx->tm_ccoef, ctx->tm_basis, ctx->tm_mom, ctx->recon, ctx->wc_basis};
  for (double* b : bufs)
    if (b) (void)hipFree(b);
  if (ctx->wtab) (void)hipFree(ctx->wtab);
  if (ctx->i0c) (void)hipFree(ctx->i0c);
  delete ctx;
  return GW_OK;
}

gw_status gw_data_inner(const gw_ctx* ctx, double* dd_out) {
  if (!ctx || !dd_out) return set_error(GW_EINVAL, "gw_data_inner: null argument");
  *dd_out = ctx->dd;
  return GW_OK;
}

gw_status loglike_batch(gw_ctx* ctx, const double* theta, int64_t n, int32_t like, int32_t marg, int32_t prec,
                        double* logl, void* stream) {
  if (!ctx) return set_error(GW_EINVAL, "loglike_batch: ctx is NULL");
  if (n < 0) return set_error(GW_EINVAL, "loglike_batch: n < 0");
  if (n > 0 && (!theta || !logl)) return set_error(GW_EINVAL, "loglike_batch: null theta or logl");
  if (like != GW_FULL && like != GW_HET) return set_error(GW_EINVAL, "loglike_batch: bad like=%d", like);
  if (marg < GW_MARG_NONE || marg > GW_MARG_PHASE_TIME) return set_error(GW_EINVAL, "loglike_batch: bad marg=%d", marg);
  if (prec != GW_PREC_FP64 && prec != GW_PREC_MIXED) return set_error(GW_EINVAL, "loglike_batch: bad prec=%d", prec);
  if (marg == GW_MARG_PHASE_DIST && ctx->n_dist <= 0)
    return set_error(GW_ESTATE, "loglike_batch: distance marginal needs a distance grid");
  if (n == 0) return GW_OK;
  hipStream_t st = (hipStream_t)stream;
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  if (like == GW_HET) return loglike_het(ctx, theta, n, marg, prec, logl, st);
  if (marg == GW_MARG_PHASE_TIME) return loglike_tmarg(ctx, theta, n, prec, logl, st);

  int tpb, nch;
  full_launch_shape(ctx, n, &tpb, &nch);
  s = ensure_buffer(&ctx->coef, &ctx->coef_cap, (int64_t)C_NCOEF * n, "coefficient workspace");
  if (s == GW_OK) s = ensure_buffer(&ctx->partial, &ctx->partial_cap, (int64_t)nch * 2 * ctx->n_det * n, "partials");
  if (s == GW_OK) s = ensure_buffer(&ctx->zbuf, &ctx->zbuf_cap, 2 * n, "marginal workspace");
  if (s != GW_OK) return s;
  const int64_t ld = n;
  s = launch_prologue(ctx, theta, n, marg, ctx->coef, ld, st);
  if (s == GW_OK) {
    const int slot = prof_begin(ctx, st, 1);
    s = launch_full(ctx, ctx->coef, ld, n, prec, tpb, nch, ctx->partial, st);
    prof_end(ctx, slot, st);
  }
  if (s == GW_OK) s = launch_epilogue(ctx, ctx->partial, nch, ctx->coef, ld, n, marg, prec, logl, st);
  return s;
}

gw_status gw_template(gw_ctx* ctx, const double* theta, int64_t n, double* h, void* stream) {
  if (!ctx) return set_error(GW_EINVAL, "gw_template: ctx is NULL");
  if (n < 0) return set_error(GW_EINVAL, "gw_template: n < 0");
  if (n > 0 && (!theta || !h)) return set_error(GW_EINVAL, "gw_template: null pointer");
  if (n == 0) return GW_OK;
  hipStream_t st = (hipStream_t)stream;
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s == GW_OK) s = ensure_buffer(&ctx->coef, &ctx->coef_cap, (int64_t)C_NCOEF * n, "coefficient workspace");
  if (s == GW_OK) s = launch_prologue(ctx, theta, n, 0, ctx->coef, n, st);
  if (s == GW_OK) s = launch_template(ctx, ctx->coef, n, n, h, st);
  return s;
}

gw_status gw_profile_enable(gw_ctx* ctx, int32_t enable) {
  if (!ctx) return set_error(GW_EINVAL, "gw_profile_enable: ctx is NULL");
  if (enable < 0 || enable > 2) return set_error(GW_EINVAL, "gw_profile_enable: enable must be 0, 1 or 2");
  ctx->prof = enable;
  return GW_OK;
}

gw_status gw_profile_read(gw_ctx* ctx, double* kernel_ms, int64_t* launches) {
  if (!ctx || !kernel_ms || !launches) return set_error(GW_EINVAL, "gw_profile_read: null argument");
  double total = 0.0;
  for (int s = 0; s < ctx->prof_used; ++s) {
    gw_status st = check_hip(hipEventSynchronize(ctx->prof_ev[2 * s + 1]), "gw_profile_read sync");
    if (st != GW_OK) return st;
    float ms = 0.0f;
    st = check_hip(hipEventElapsedTime(&ms, ctx->prof_ev[2 * s], ctx->prof_ev[2 * s + 1]), "gw_profile_read");
    if (st != GW_OK) return st;
    total += ms;
  }
  *kernel_ms = total;
  *launches = ctx->prof_used;
  ctx->prof_used = 0;
  return GW_OK;
}

// Tuning knobs of the full-band kernel (0 restores the heuristic).
gw_status gw_set_full_shape(gw_ctx* ctx, int32_t tpb, int32_t n_chunks) {
  if (!ctx) return set_error(GW_EINVAL, "gw_set_full_shape: ctx is NULL");
  if (tpb != 0 && tpb != 64 && tpb != 128 && tpb != 256)
    return set_error(GW_EINVAL, "gw_set_full_shape: tpb must be 0, 64, 128 or 256");
  if (n_chunks < 0) return set_error(GW_EINVAL, "gw_set_full_shape: n_chunks < 0");
  ctx->full_tpb = tpb;
  ctx->full_chunks = n_chunks;
  ++ctx->gen;
  return GW_OK;
}

gw_status gw_set_full_kernel(gw_ctx* ctx, int32_t kind) {
  if (!ctx) return set_error(GW_EINVAL, "gw_set_full_kernel: ctx is NULL");
  if (kind < 0 || kind > 2) return set_error(GW_EINVAL, "gw_set_full_kernel: kind must be 0, 1 or 2");
  ctx->full_kernel = kind;
  ++ctx->gen;
  return GW_OK;
}

gw_status gw_phasor_gain(const gw_ctx* ctx, double* re, double* im) {
  if (!ctx || !re || !im) return set_error(GW_EINVAL, "gw_phasor_gain: null argument");
  *re = ctx->pgain_re;
  *im = ctx->pgain_im;
  return GW_OK;
}

gw_status gw_full_info(const gw_ctx* ctx, int32_t* mom_blk) {
  if (!ctx || !mom_blk) return set_error(GW_EINVAL, "gw_full_info: null argument");
  *mom_blk = ctx->mom_blk;
  return GW_OK;
}

}  // extern "C"
