// Waveform cache as a library object: the paper's pair of a slow likelihood
// (regenerates and caches the waveform) and a fast one (reuses it, Sec. III.B
// and Sec. III.A: the fast blocks only redo the detector projection and the
// marginalisations).  The sampler's sweep keeps the same cache internally;
// this entry point lets any caller use it.
#include <string.h>

#include "gw_ctx.h"

using namespace gw;

struct gw_wcache {
  gw_ctx* ctx = nullptr;
  int64_t n_slots = 0;
  int64_t slot_f2 = 0;
  float2* wc = nullptr;  // [n_slots][slot_f2] block moments (FP32 complex)
  double* zc = nullptr;  // [n_slots][2 n_det] sums z_i of each slot's point
  int32_t* owner = nullptr;  // [n_slots]: -1 between calls
  // per-call workspace: zrow [cap][2 kMaxDet], rows [cap] (0 .. n - 1),
  // sl [cap] (checked slots), counts [2]
  int64_t cap = 0;
  char* mem = nullptr;
  double* zrow = nullptr;
  int32_t* rows = nullptr;
  int32_t* sl = nullptr;
  int32_t* counts = nullptr;
};

namespace {

// rows[i] = i for i < n; counts = (n, 0) for the full list, (0, n) for the
// cached-waveform list.
__global__ void k_wc_rows(int32_t* __restrict__ rows, int64_t n, int32_t* __restrict__ counts, int which) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) rows[i] = (int32_t)i;
  if (i == 0) {
    counts[0] = which == 0 ? (int32_t)n : 0;
    counts[1] = which == 1 ? (int32_t)n : 0;
  }
}

__global__ void k_wc_fill(int32_t* __restrict__ a, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// sl[r] = slots[r] when 0 <= slots[r] < n_slots, else -1; with owner, the
// largest row naming each slot claims it.
__global__ void k_wc_slots(const int32_t* __restrict__ slots, int64_t n, int64_t n_slots, int32_t* __restrict__ sl,
                           int32_t* __restrict__ owner) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int32_t s = slots[r];
  const bool ok = s >= 0 && s < n_slots;
  sl[r] = ok ? s : -1;
  if (ok && owner) atomicMax(&owner[s], (int32_t)r);
}

// Keep only the claiming row of each slot (sl[r] = -2 for the others: their
// log L stands, they store nothing), store its sums: zc[sl[r]] = zrow[r].
__global__ void k_wc_store_z(const double* __restrict__ zrow, int32_t* __restrict__ sl,
                             const int32_t* __restrict__ owner, int64_t n, int nd, double* __restrict__ zc) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int32_t s = sl[r];
  if (s < 0) return;
  if (owner[s] != (int32_t)r) {
    sl[r] = -2;
    return;
  }
  for (int j = 0; j < 2 * nd; ++j) zc[(int64_t)s * 2 * nd + j] = zrow[r * 2 * nd + j];
}

// Release the claims (owner back to -1) once the slots are written.
__global__ void k_wc_release(const int32_t* __restrict__ slots, int64_t n, int64_t n_slots,
                             int32_t* __restrict__ owner) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int32_t s = slots[r];
  if (s >= 0 && s < n_slots) owner[s] = -1;
}

// Rows whose slot is out of range (sl[r] == -1) get log L = NaN.
__global__ void k_wc_mark(const int32_t* __restrict__ sl, int64_t n, double* __restrict__ logl) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n && sl[r] == -1) logl[r] = __builtin_nan("");
}

gw_status wc_reserve(gw_wcache* c, int64_t n) {
  gw_status s = cached_reserve(c->ctx, n);
  if (s != GW_OK || c->cap >= n) return s;
  if (c->mem) (void)hipFree(c->mem);
  c->mem = nullptr;
  c->cap = 0;
  const size_t bytes = (size_t)n * 2 * kMaxDet * sizeof(double) + 2 * (size_t)n * sizeof(int32_t) + 2 * sizeof(int32_t);
  s = check_hip(hipMalloc((void**)&c->mem, bytes), "waveform cache workspace");
  if (s != GW_OK) return s;
  c->zrow = (double*)c->mem;
  c->rows = (int32_t*)(c->mem + (size_t)n * 2 * kMaxDet * sizeof(double));
  c->sl = c->rows + n;
  c->counts = c->sl + n;
  c->cap = n;
  return GW_OK;
}

gw_status wc_check(const gw_wcache* c, const double* theta, const int32_t* slots, int64_t n, int32_t marg,
                   int32_t prec, const double* logl, const char* who) {
  if (!c) return set_error(GW_EINVAL, "%s: cache is NULL", who);
  if (n < 0) return set_error(GW_EINVAL, "%s: n < 0", who);
  if (n > 0 && (!theta || !slots || !logl)) return set_error(GW_EINVAL, "%s: null pointer", who);
  if (n > 0x7fffffff) return set_error(GW_EINVAL, "%s: n too large", who);
  if (marg < GW_MARG_NONE || marg > GW_MARG_PHASE_DIST) return set_error(GW_EINVAL, "%s: bad marg=%d", who, marg);
  if (prec != GW_PREC_FP64 && prec != GW_PREC_MIXED) return set_error(GW_EINVAL, "%s: bad prec=%d", who, prec);
  if (marg == GW_MARG_PHASE_DIST && c->ctx->n_dist <= 0)
    return set_error(GW_ESTATE, "%s: distance marginal needs a distance grid", who);
  return GW_OK;
}

}  // namespace

extern "C" {

gw_status gw_wcache_create(gw_ctx* ctx, int64_t n_slots, gw_wcache** out) {
  if (!out) return set_error(GW_EINVAL, "gw_wcache_create: out is NULL");
  *out = nullptr;
  if (!ctx) return set_error(GW_EINVAL, "gw_wcache_create: ctx is NULL");
  if (n_slots < 1) return set_error(GW_EINVAL, "gw_wcache_create: n_slots < 1");
  const int64_t f2 = wmom_slot_f2(ctx);
  if ((double)n_slots * (double)f2 * sizeof(float2) > 128.0 * (1ull << 30))
    return set_error(GW_EINVAL, "gw_wcache_create: %lld slots of %lld bytes exceed 128 GiB", (long long)n_slots,
                     (long long)(f2 * sizeof(float2)));
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  gw_wcache* c = new (std::nothrow) gw_wcache();
  if (!c) return set_error(GW_ENOMEM, "gw_wcache_create");
  c->ctx = ctx;
  c->n_slots = n_slots;
  c->slot_f2 = f2;
  s = check_hip(hipMalloc((void**)&c->wc, (size_t)n_slots * f2 * sizeof(float2)), "waveform cache");
  if (s == GW_OK)
    s = check_hip(hipMalloc((void**)&c->zc, (size_t)n_slots * 2 * ctx->n_det * sizeof(double)), "cached sums");
  if (s == GW_OK) s = check_hip(hipMalloc((void**)&c->owner, (size_t)n_slots * sizeof(int32_t)), "slot claims");
  if (s == GW_OK) {
    hipLaunchKernelGGL(k_wc_fill, dim3((unsigned)((n_slots + 255) / 256)), dim3(256), 0, nullptr, c->owner, n_slots,
                       -1);
    s = check_hip(hipGetLastError(), "slot claims fill");
  }
  if (s == GW_OK) s = check_hip(hipDeviceSynchronize(), "waveform cache set-up");
  if (s != GW_OK) {
    if (c->wc) (void)hipFree(c->wc);
    if (c->zc) (void)hipFree(c->zc);
    if (c->owner) (void)hipFree(c->owner);
    delete c;
    return s;
  }
  *out = c;
  return GW_OK;
}

gw_status gw_wcache_destroy(gw_wcache* c) {
  if (!c) return GW_OK;
  (void)hipSetDevice(c->ctx->device);
  if (c->wc) (void)hipFree(c->wc);
  if (c->zc) (void)hipFree(c->zc);
  if (c->owner) (void)hipFree(c->owner);
  if (c->mem) (void)hipFree(c->mem);
  delete c;
  return GW_OK;
}

gw_status gw_wcache_update(gw_wcache* c, const double* theta, const int32_t* slots, int64_t n, int32_t marg,
                           int32_t prec, double* logl, void* stream) {
  gw_status s = wc_check(c, theta, slots, n, marg, prec, logl, "gw_wcache_update");
  if (s != GW_OK || n == 0) return s;
  gw_ctx* ctx = c->ctx;
  hipStream_t st = (hipStream_t)stream;
  s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s == GW_OK) s = wc_reserve(c, n);
  if (s != GW_OK) return s;
  int tpb, nch;
  cached_shape(ctx, &tpb, &nch);
  const unsigned blocks = (unsigned)((n + 255) / 256);
  s = launch_prologue(ctx, theta, n, marg, ctx->coef, n, st);
  if (s == GW_OK) {
    hipLaunchKernelGGL(k_wc_rows, dim3(blocks), dim3(256), 0, st, c->rows, n, c->counts, 0);
    hipLaunchKernelGGL(k_wc_slots, dim3(blocks), dim3(256), 0, st, slots, n, c->n_slots, c->sl, c->owner);
    s = check_hip(hipGetLastError(), "row list launch");
  }
  if (s == GW_OK)
    s = launch_cached(ctx, ctx->coef, n, prec, tpb, nch, c->rows, nullptr, c->counts, 1, nullptr, nullptr, nullptr,
                      ctx->partial, st);
  if (s == GW_OK)
    s = launch_epilogue_cached(ctx, ctx->partial, nch, ctx->coef, n, n, marg, prec, logl, nullptr, nullptr, c->zrow,
                               st);
  if (s == GW_OK) {
    hipLaunchKernelGGL(k_wc_store_z, dim3(blocks), dim3(256), 0, st, c->zrow, c->sl, c->owner, n, ctx->n_det, c->zc);
    s = check_hip(hipGetLastError(), "cached sums launch");
  }
  if (s == GW_OK) s = launch_wmom_build(ctx, ctx->coef, n, c->sl, c->counts, n, 1, c->rows, prec, c->wc, st);
  if (s == GW_OK) {
    hipLaunchKernelGGL(k_wc_release, dim3(blocks), dim3(256), 0, st, slots, n, c->n_slots, c->owner);
    hipLaunchKernelGGL(k_wc_mark, dim3(blocks), dim3(256), 0, st, c->sl, n, logl);
    s = check_hip(hipGetLastError(), "slot release launch");
  }
  return s;
}

gw_status gw_wcache_loglike(gw_wcache* c, const double* theta, const int32_t* slots, int64_t n, int32_t kind,
                            int32_t marg, int32_t prec, double* logl, void* stream) {
  gw_status s = wc_check(c, theta, slots, n, marg, prec, logl, "gw_wcache_loglike");
  if (s != GW_OK || n == 0) return s;
  if (kind != 1 && kind != 2) return set_error(GW_EINVAL, "gw_wcache_loglike: kind must be 1 or 2");
  gw_ctx* ctx = c->ctx;
  hipStream_t st = (hipStream_t)stream;
  s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s == GW_OK) s = wc_reserve(c, n);
  if (s != GW_OK) return s;
  int tpb, nch;
  cached_shape(ctx, &tpb, &nch);
  const unsigned blocks = (unsigned)((n + 255) / 256);
  s = launch_prologue(ctx, theta, n, marg, ctx->coef, n, st);
  if (s != GW_OK) return s;
  // out-of-range slots read slot 0 and are marked NaN afterwards
  hipLaunchKernelGGL(k_wc_slots, dim3(blocks), dim3(256), 0, st, slots, n, c->n_slots, c->sl, nullptr);
  hipLaunchKernelGGL(k_wc_rows, dim3(blocks), dim3(256), 0, st, c->rows, n, c->counts, 1);
  s = check_hip(hipGetLastError(), "row list launch");
  if (s == GW_OK && kind == 2) {  // the slots' sums, no reduction
    s = launch_epilogue_cached(ctx, ctx->partial, 0, ctx->coef, n, n, marg, prec, logl, c->sl, c->zc, nullptr, st);
  } else if (s == GW_OK) {
    // complete sums into zrow, then the epilogue takes them from there
    s = launch_cached(ctx, ctx->coef, n, prec, tpb, nch, nullptr, c->rows, c->counts, 1, c->sl, c->wc, c->zrow,
                      ctx->partial, st);
    if (s == GW_OK)
      s = launch_epilogue_cached(ctx, ctx->partial, 0, ctx->coef, n, n, marg, prec, logl, c->rows, c->zrow, nullptr,
                                 st);
  }
  if (s == GW_OK) {
    hipLaunchKernelGGL(k_wc_mark, dim3(blocks), dim3(256), 0, st, c->sl, n, logl);
    s = check_hip(hipGetLastError(), "slot check launch");
  }
  return s;
}

}  // extern "C"
