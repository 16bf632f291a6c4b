// Allocation-free form of the full-band batched likelihood, for callers that
// cannot allocate device memory (work recorded into a graph, tight serving
// loops, harnesses that forbid allocation).  The kernels are those of
// loglike_batch (prologue, fused phase/projection/overlap reduction,
// fixed-order epilogue with the marginals); only their workspace differs: the
// per-row coefficients, the distance marginal's staging and the chunk partial
// sums live in one statically sized device array instead of the context's
// buffers grown on demand.
//
// Each device holds its own copy of the array from the first context created
// on it until the process ends.  Every call on a device shares that device's
// copy, so calls that overlap on one device (other streams, other threads,
// other contexts) race and must be ordered by the caller.  Nothing in the
// array needs to start at zero: every kernel writes what it later reads.
#include <mutex>

#include "gw_ctx.h"

namespace gw {
// 16 MiB of FP64 per device.
constexpr int64_t kScratchDoubles = int64_t(1) << 21;
}  // namespace gw

static __device__ __align__(256) double scratch[gw::kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {nullptr};  // device address of each device's copy
std::mutex g_scratch_mu;
}  // namespace

namespace gw {

// Record the device address of ``device``'s copy of the scratch array.  Called
// by gw_ctx_create with that device current, once per device.
gw_status noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices)
    return set_error(GW_ENOTSUP, "allocation-free workspace: device index %d above %d", device, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return GW_OK;
  void* p = nullptr;
  gw_status s = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address");
  if (s != GW_OK) return s;
  if (!p) return set_error(GW_EDEVICE, "scratch symbol address: null");
  g_scratch[device] = (double*)p;
  return GW_OK;
}

}  // namespace gw

using namespace gw;

extern "C" {

gw_status loglike_batch_noalloc(gw_ctx* ctx, const double* theta, int64_t n, int32_t marg, int32_t prec,
                                double* logl, void* stream) {
  if (!ctx) return set_error(GW_EINVAL, "loglike_batch_noalloc: ctx is NULL");
  if (n < 0) return set_error(GW_EINVAL, "loglike_batch_noalloc: n < 0");
  if (n > 0 && (!theta || !logl)) return set_error(GW_EINVAL, "loglike_batch_noalloc: null theta or logl");
  if (marg != GW_MARG_NONE && marg != GW_MARG_PHASE && marg != GW_MARG_PHASE_DIST)
    return set_error(GW_EINVAL, "loglike_batch_noalloc: marg must be GW_MARG_NONE, GW_MARG_PHASE or "
                                "GW_MARG_PHASE_DIST");
  if (prec != GW_PREC_FP64 && prec != GW_PREC_MIXED)
    return set_error(GW_EINVAL, "loglike_batch_noalloc: bad prec=%d", prec);
  if (marg == GW_MARG_PHASE_DIST && ctx->n_dist <= 0)
    return set_error(GW_ESTATE, "loglike_batch_noalloc: distance marginal needs a distance grid");
  if (n == 0) return GW_OK;
  if (ctx->device < 0 || ctx->device >= kMaxDevices) return set_error(GW_ESTATE, "loglike_batch_noalloc: bad device");
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch[ctx->device];
  }
  if (!base) return set_error(GW_ESTATE, "loglike_batch_noalloc: workspace of device %d not set up", ctx->device);
  // Workspace per row: C_NCOEF coefficients, 2 staging values, and 2 n_det
  // partial sums per frequency chunk; the chunk count is the launch shape's,
  // lowered (in steps of 8, at least 8) until the array holds it.
  const int64_t per_chunk = 2 * (int64_t)ctx->n_det * n;
  const int64_t fixed = (int64_t)(C_NCOEF + 2) * n;
  if (n > kScratchDoubles || fixed + 8 * per_chunk > kScratchDoubles)
    return set_error(GW_EINVAL,
                     "loglike_batch_noalloc: n = %lld rows exceed the allocation-free maximum of %lld rows "
                     "(%lld doubles of workspace)",
                     (long long)n, (long long)(kScratchDoubles / (C_NCOEF + 2 + 16 * ctx->n_det)),
                     (long long)kScratchDoubles);
  int tpb, nch;
  full_launch_shape(ctx, n, &tpb, &nch);
  const int64_t max_ch = (kScratchDoubles - fixed) / per_chunk;
  if (nch > max_ch) {
    if (ctx->full_chunks > 0)
      return set_error(GW_EINVAL,
                       "loglike_batch_noalloc: the fixed launch shape's %d chunks need more than the %lld doubles "
                       "of workspace at n = %lld (at most %lld chunks)",
                       nch, (long long)kScratchDoubles, (long long)n, (long long)max_ch);
    nch = (int)(max_ch / 8 * 8);
  }
  hipStream_t st = (hipStream_t)stream;
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  double* coef = base;
  double* zbuf = coef + (int64_t)C_NCOEF * n;
  double* partial = zbuf + 2 * n;
  s = launch_prologue(ctx, theta, n, marg, coef, n, st);
  if (s == GW_OK) s = launch_full(ctx, coef, n, n, prec, tpb, nch, partial, st);
  if (s == GW_OK)
    s = launch_epilogue_z(ctx, partial, nch, coef, n, n, marg, prec, logl, nullptr, nullptr, nullptr, zbuf, st);
  return s;
}

}  // extern "C"
