// Constrained hit-and-run slice step over k chains for one Gibbs block
// (Sec. II.C and III.B, Eq. block_cprior).  Each chain moves its block of
// unit-cube coordinates along t -> x + t d with d = L u (u a random unit
// vector, L the Cholesky factor of the block covariance), stepping the
// bracket out while its ends satisfy log L > log L*, then shrinking it until a
// point inside the constraint is found.  Chains advance in rounds: a propose
// kernel writes every chain's candidate points as parameter vectors, the
// batched likelihood evaluates them all, and an update kernel moves each
// chain's state machine; the host checks for completion every few rounds.
#include <math.h>
#include <string.h>

#include <vector>

#include "gw_ctx.h"

namespace gw {

constexpr int kSliceDim = 11;
constexpr int kMaxBlock = 4;
constexpr int kUniFixed = 5;  // 4 direction + 1 bracket offset

struct SliceParams {
  int32_t block[kMaxBlock];
  double chol[kMaxBlock * kMaxBlock];
  int32_t bd;
  double w;
  double logl_star;
  int32_t max_out, max_shrink;
  uint64_t seed, counter;
  const double* uniforms;  // [k][kUniFixed + max_shrink] or null
  int64_t k;
};

// Parameters of one call as a device block, so that a captured graph of the
// round loop reads them at replay time instead of baking them in.
struct SliceDev {
  SliceParams P;
  double* x;
  double* logl;
};

// Per-chain state (structure of arrays inside one device allocation).
struct SliceState {
  double* t_lo;
  double* t_hi;
  double* d;        // [k][kMaxBlock]
  double* cand_t;   // [k][2]
  int32_t* flags;   // [k]: bit0 lo stepping, bit1 hi stepping, bit2 done, bit3 kept (cap hit)
  int32_t* n_out;   // [k][2]
  int32_t* n_shrink;
  int32_t* n_evals;
  int32_t* slot_ok;  // [k][2]: candidate inside the cube and needs a likelihood
  int32_t* n_active;
};

// Philox4x64-10 (Salmon, Moraes, Dror & Shaw 2011).
__device__ inline void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

// Uniform j of chain c: explicit table, or Philox word j % 4 of counter
// (counter_base, c, j / 4, 0) under key (seed, 0), mapped to (0, 1).
__device__ inline double slice_uniform(const SliceParams& P, int64_t c, int j) {
  if (P.uniforms) return P.uniforms[c * (kUniFixed + P.max_shrink) + j];
  uint64_t ctr[4] = {P.counter, (uint64_t)c, (uint64_t)(j >> 2), 0ull};
  philox4x64(ctr, P.seed, 0ull);
  return ((double)(ctr[j & 3] >> 11) + 0.5) * 1.1102230246251565404e-16;  // 2^-53
}

// Unit cube -> 13-column parameter vector (d_L = 1, phi_c = 0; both are
// marginalised by the modes slice_step accepts).
__device__ inline void prior_transform(const double* u, double* th) {
  const double lo[6] = {1.1, 0.5, -0.05, -0.05, 0.0, 0.0};
  const double hi[6] = {1.4, 1.0, 0.05, 0.05, 5000.0, 5000.0};
#pragma unroll
  for (int j = 0; j < 6; ++j) th[j] = lo[j] + (hi[j] - lo[j]) * u[j];
  th[6] = 1.0;
  th[7] = acos(1.0 - 2.0 * u[6]);
  th[8] = kTwoPi * u[7];
  th[9] = asin(2.0 * u[8] - 1.0);
  th[10] = kPi * u[9];
  th[11] = 0.0;
  th[12] = -0.1 + 0.2 * u[10];
}

__global__ void k_slice_init(SliceParams P, SliceState S) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.k) return;
  double u[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) u[j] = slice_uniform(P, c, j);
  const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
  double s0, c0, s1, c1;
  sincos(kTwoPi * u[1], &s0, &c0);
  sincos(kTwoPi * u[3], &s1, &c1);
  double z[4] = {r0 * c0, r0 * s0, r1 * c1, r1 * s1};
  double nrm = 0.0;
  for (int j = 0; j < P.bd; ++j) nrm += z[j] * z[j];
  nrm = sqrt(nrm);
  for (int a = 0; a < kMaxBlock; ++a) {
    double v = 0.0;
    for (int b = 0; b < P.bd; ++b)
      if (a < P.bd) v += P.chol[a * kMaxBlock + b] * (z[b] / nrm);
    S.d[c * kMaxBlock + a] = a < P.bd ? v : 0.0;
  }
  const double off = slice_uniform(P, c, 4);
  S.t_lo[c] = -off * P.w;
  S.t_hi[c] = (1.0 - off) * P.w;
  S.flags[c] = P.max_out > 0 ? 3 : 0;
  S.n_out[2 * c] = 0;
  S.n_out[2 * c + 1] = 0;
  S.n_shrink[c] = 0;
  S.n_evals[c] = 0;
}

__device__ inline bool make_point(const SliceParams& P, const SliceState& S, const double* x0, int64_t c, double t,
                                  double* u) {
  for (int j = 0; j < kSliceDim; ++j) u[j] = x0[c * kSliceDim + j];
  bool inside = true;
  for (int a = 0; a < P.bd; ++a) {
    const int j = P.block[a];
    const double v = x0[c * kSliceDim + j] + t * S.d[c * kMaxBlock + a];
    inside = inside && v >= 0.0 && v <= 1.0;
    u[j] = v;
  }
  return inside;
}

// Write the candidates of every chain that is still moving: the two bracket
// ends while stepping out, else one shrink draw (points outside the cube
// count as rejections immediately, without a likelihood call).
__global__ void k_slice_set(SliceDev* D, SliceParams P, double* x, double* logl) {
  D->P = P;
  D->x = x;
  D->logl = logl;
}

__global__ void k_slice_propose(const SliceDev* __restrict__ D, SliceState S, double* __restrict__ cand) {
  const SliceParams& P = D->P;
  const double* __restrict__ x0 = D->x;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) *S.n_active = 0;
  if (c >= P.k) return;
  int fl = S.flags[c];
  double u[kSliceDim];
  int ok[2] = {0, 0};
  if (!(fl & 4)) {
    if (fl & 3) {
      for (int side = 0; side < 2; ++side) {
        if (!(fl & (1 << side))) continue;
        const double t = side == 0 ? S.t_lo[c] : S.t_hi[c];
        if (make_point(P, S, x0, c, t, u)) {
          prior_transform(u, cand + (2 * c + side) * 13);
          S.cand_t[2 * c + side] = t;
          ok[side] = 1;
        } else {
          fl &= ~(1 << side);  // outside the cube: this side stops here
        }
      }
    }
    if (!(fl & 3)) {
      // shrinking: draw until a point lies in the cube (no likelihood needed
      // for the others) or the cap is reached
      while (S.n_shrink[c] < P.max_shrink) {
        const double v = slice_uniform(P, c, kUniFixed + S.n_shrink[c]);
        const double t = S.t_lo[c] + v * (S.t_hi[c] - S.t_lo[c]);
        if (make_point(P, S, x0, c, t, u)) {
          prior_transform(u, cand + 2 * c * 13);
          S.cand_t[2 * c] = t;
          ok[0] = 1;
          break;
        }
        if (t < 0.0) S.t_lo[c] = t;
        else S.t_hi[c] = t;
        S.n_shrink[c] += 1;
      }
      if (!ok[0]) fl |= 12;  // cap reached: keep the old point
    }
  }
  // rows that need no likelihood get an unphysical vector (cheap -inf)
  for (int side = 0; side < 2; ++side)
    if (!ok[side]) {
      double* th = cand + (2 * c + side) * 13;
      for (int j = 0; j < 13; ++j) th[j] = 0.0;
      th[1] = -1.0;
    }
  S.slot_ok[2 * c] = ok[0];
  S.slot_ok[2 * c + 1] = ok[1];
  S.flags[c] = fl;
}

__global__ void k_slice_update(const SliceDev* __restrict__ D, SliceState S, const double* __restrict__ cand_logl) {
  const SliceParams& P = D->P;
  double* __restrict__ x = D->x;
  double* __restrict__ logl = D->logl;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.k) return;
  int fl = S.flags[c];
  if (fl & 4) return;
  const bool stepping = (fl & 3) != 0;
  if (stepping) {
    for (int side = 0; side < 2; ++side) {
      if (!S.slot_ok[2 * c + side]) continue;
      S.n_evals[c] += 1;
      const bool in = cand_logl[2 * c + side] > P.logl_star;
      int no = S.n_out[2 * c + side];
      if (in && no < P.max_out) {
        if (side == 0) S.t_lo[c] -= P.w;
        else S.t_hi[c] += P.w;
        no += 1;
        S.n_out[2 * c + side] = no;
        if (no >= P.max_out) fl &= ~(1 << side);
      } else {
        fl &= ~(1 << side);
      }
    }
  } else if (S.slot_ok[2 * c]) {
    S.n_evals[c] += 1;
    const double v = cand_logl[2 * c];
    const double t = S.cand_t[2 * c];
    if (v > P.logl_star) {
      for (int a = 0; a < P.bd; ++a) {
        const int j = P.block[a];
        x[c * kSliceDim + j] += t * S.d[c * kMaxBlock + a];
      }
      logl[c] = v;
      fl |= 4;
    } else {
      if (t < 0.0) S.t_lo[c] = t;
      else S.t_hi[c] = t;
      S.n_shrink[c] += 1;
      if (S.n_shrink[c] >= P.max_shrink) fl |= 12;
    }
  }
  S.flags[c] = fl;
  if (!(fl & 4)) atomicAdd(S.n_active, 1);
}

__global__ void k_prior_transform(const double* __restrict__ x, int64_t n, double* __restrict__ theta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) prior_transform(x + i * kSliceDim, theta + i * 13);
}

__global__ void k_slice_finish(SliceParams P, SliceState S, int32_t* n_evals, int32_t* status) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.k) return;
  if (n_evals) n_evals[c] = S.n_evals[c];
  if (status) status[c] = (S.flags[c] & 8) ? 1 : 0;
}

}  // namespace gw

using namespace gw;

// What a captured round group bakes in: any change means a new capture.
struct SliceGraphKey {
  int64_t k;
  int32_t like, marg, prec;
  const void *ws_mem, *coef, *partial, *zbuf, *het;
  int32_t het_wpb, het_grid, het_ech, full_tpb, full_chunks, full_kernel;
  bool operator==(const SliceGraphKey& o) const { return memcmp(this, &o, sizeof(*this)) == 0; }
};

struct gw_slice_ws {
  int64_t cap = 0;
  void* mem = nullptr;
  double* cand = nullptr;       // [2k][13]
  double* cand_logl = nullptr;  // [2k]
  int32_t* h_active = nullptr;  // pinned host
  SliceState S{};
  SliceDev* dev = nullptr;      // device parameter block
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  SliceGraphKey key{};
  bool have_graph = false;
};

static gw_status slice_ws(gw_ctx* ctx, int64_t k, gw_slice_ws** out);

// Capture one round group into a graph (re-captured when anything it bakes in
// changes) on the workspace's own capture stream.  Buffers the likelihood
// would grow are reserved first: no allocation may happen during capture.
template <class Group>
static gw_status slice_graph(gw_ctx* ctx, gw_slice_ws* ws, const gw_slice_args* a, Group group) {
  const int64_t n = 2 * a->k;
  gw_status s = a->like == GW_HET ? het_reserve(ctx, n) : full_reserve(ctx, n);
  if (s != GW_OK) return s;
  SliceGraphKey key;
  memset(&key, 0, sizeof(key));
  key.k = a->k;
  key.like = a->like;
  key.marg = a->marg;
  key.prec = a->prec;
  key.ws_mem = ws->mem;
  key.coef = ctx->coef;
  key.partial = ctx->partial;
  key.zbuf = ctx->zbuf;
  key.het = ctx->het;
  het_shape_key(ctx, &key.het_wpb, &key.het_grid, &key.het_ech);
  key.full_tpb = ctx->full_tpb;
  key.full_chunks = ctx->full_chunks;
  key.full_kernel = ctx->full_kernel;
  if (ws->have_graph && ws->key == key) return GW_OK;
  if (ws->exec) (void)hipGraphExecDestroy(ws->exec);
  if (ws->graph) (void)hipGraphDestroy(ws->graph);
  ws->exec = nullptr;
  ws->graph = nullptr;
  ws->have_graph = false;
  if (!ws->cap_stream) {
    s = check_hip(hipStreamCreateWithFlags(&ws->cap_stream, hipStreamNonBlocking), "capture stream");
    if (s != GW_OK) return s;
  }
  const bool prof = ctx->prof;
  ctx->prof = false;  // no timing events inside the graph
  s = check_hip(hipStreamBeginCapture(ws->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  gw_status g = GW_OK;
  if (s == GW_OK) g = group(ws->cap_stream);
  hipGraph_t graph = nullptr;
  if (s == GW_OK) s = check_hip(hipStreamEndCapture(ws->cap_stream, &graph), "end capture");
  ctx->prof = prof;
  if (s == GW_OK && g != GW_OK) s = g;
  if (s == GW_OK) s = check_hip(hipGraphInstantiate(&ws->exec, graph, nullptr, nullptr, 0), "graph instantiate");
  if (s != GW_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    ws->exec = nullptr;
    return s;
  }
  ws->graph = graph;
  ws->key = key;
  ws->have_graph = true;
  return GW_OK;
}

extern "C" {

gw_status slice_step(gw_ctx* ctx, const gw_slice_args* a, void* stream) {
  if (!ctx || !a) return set_error(GW_EINVAL, "slice_step: null argument");
  if (a->k < 0) return set_error(GW_EINVAL, "slice_step: k < 0");
  if (a->k == 0) return GW_OK;
  if (!a->x || !a->logl || !a->block || !a->chol) return set_error(GW_EINVAL, "slice_step: null pointer");
  if (a->block_dim < 1 || a->block_dim > kMaxBlock) return set_error(GW_EINVAL, "slice_step: block_dim 1..4");
  for (int i = 0; i < a->block_dim; ++i) {
    if (a->block[i] < 0 || a->block[i] >= kSliceDim) return set_error(GW_EINVAL, "slice_step: block index 0..10");
    for (int j = 0; j < i; ++j)
      if (a->block[j] == a->block[i]) return set_error(GW_EINVAL, "slice_step: repeated block index");
  }
  if (!(a->w > 0.0) || !isfinite(a->w)) return set_error(GW_EINVAL, "slice_step: w must be > 0");
  if (a->max_out < 0 || a->max_shrink < 1 || a->max_shrink > 10000)
    return set_error(GW_EINVAL, "slice_step: max_out >= 0, max_shrink 1..10000");
  if (a->marg == GW_MARG_NONE)
    return set_error(GW_ENOTSUP, "slice_step: the 11-D sampler needs phi_c and d_L marginalised (marg=2)");
  if (a->marg != GW_MARG_PHASE_DIST) return set_error(GW_ENOTSUP, "slice_step: marg must be GW_MARG_PHASE_DIST");
  if (a->like == GW_HET && !ctx->het) return set_error(GW_ESTATE, "slice_step: heterodyne_setup has not been called");
  hipStream_t st = (hipStream_t)stream;
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  gw_slice_ws* ws = nullptr;
  s = slice_ws(ctx, a->k, &ws);
  if (s != GW_OK) return s;

  SliceParams P{};
  for (int i = 0; i < kMaxBlock; ++i) P.block[i] = i < a->block_dim ? a->block[i] : 0;
  for (int i = 0; i < kMaxBlock * kMaxBlock; ++i) P.chol[i] = 0.0;
  for (int i = 0; i < a->block_dim; ++i)
    for (int j = 0; j <= i; ++j) P.chol[i * kMaxBlock + j] = a->chol[i * a->block_dim + j];
  P.bd = a->block_dim;
  P.w = a->w;
  P.logl_star = a->logl_star;
  P.max_out = a->max_out;
  P.max_shrink = a->max_shrink;
  P.seed = a->seed;
  P.counter = a->counter;
  P.uniforms = a->uniforms;
  P.k = a->k;
  const int tpb = 256;
  const unsigned blocks = (unsigned)((a->k + tpb - 1) / tpb);
  hipLaunchKernelGGL(k_slice_set, dim3(1), dim3(1), 0, st, ws->dev, P, a->x, a->logl);
  hipLaunchKernelGGL(k_slice_init, dim3(blocks), dim3(tpb), 0, st, P, ws->S);
  s = check_hip(hipGetLastError(), "slice init launch");
  // One group = 4 rounds of (propose, batched likelihood, update); after a
  // group the host reads the number of chains still moving.  Stepping out
  // takes at most max_out + 1 rounds per side (both sides in parallel) and
  // shrinking at most max_shrink, so after max_rounds every chain is done and
  // further rounds change nothing.
  const int max_rounds = a->max_out + 1 + a->max_shrink + 1;
  auto group = [&](hipStream_t gs) -> gw_status {
    gw_status g = GW_OK;
    for (int r = 0; r < 4 && g == GW_OK; ++r) {
      hipLaunchKernelGGL(k_slice_propose, dim3(blocks), dim3(tpb), 0, gs, (const SliceDev*)ws->dev, ws->S, ws->cand);
      g = check_hip(hipGetLastError(), "slice propose launch");
      if (g == GW_OK) g = loglike_batch(ctx, ws->cand, 2 * a->k, a->like, a->marg, a->prec, ws->cand_logl, gs);
      if (g == GW_OK) {
        hipLaunchKernelGGL(k_slice_update, dim3(blocks), dim3(tpb), 0, gs, (const SliceDev*)ws->dev, ws->S,
                           (const double*)ws->cand_logl);
        g = check_hip(hipGetLastError(), "slice update launch");
      }
    }
    return g;
  };
  if (s == GW_OK && a->use_graph) s = slice_graph(ctx, ws, a, group);
  for (int rounds = 0; s == GW_OK && rounds < max_rounds; rounds += 4) {
    if (a->use_graph) s = check_hip(hipGraphLaunch(ws->exec, st), "slice graph launch");
    else s = group(st);
    if (s != GW_OK) break;
    s = check_hip(hipMemcpyAsync(ws->h_active, ws->S.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy");
    if (s == GW_OK) s = check_hip(hipStreamSynchronize(st), "slice round sync");
    if (s == GW_OK && *ws->h_active == 0) break;
  }
  if (s != GW_OK) return s;
  hipLaunchKernelGGL(k_slice_finish, dim3(blocks), dim3(tpb), 0, st, P, ws->S, a->n_evals, a->status);
  return check_hip(hipGetLastError(), "slice finish launch");
}

gw_status gw_prior_transform(gw_ctx* ctx, const double* x, int64_t n, double* theta, void* stream) {
  if (!ctx) return set_error(GW_EINVAL, "gw_prior_transform: ctx is NULL");
  if (n < 0) return set_error(GW_EINVAL, "gw_prior_transform: n < 0");
  if (n == 0) return GW_OK;
  if (!x || !theta) return set_error(GW_EINVAL, "gw_prior_transform: null pointer");
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  hipLaunchKernelGGL(k_prior_transform, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, x, n,
                     theta);
  return check_hip(hipGetLastError(), "prior transform launch");
}

}  // extern "C"

static gw_status slice_ws(gw_ctx* ctx, int64_t k, gw_slice_ws** out) {
  gw_slice_ws*& ws = ctx->slice;
  if (!ws) {
    ws = new (std::nothrow) gw_slice_ws();
    if (!ws) return set_error(GW_ENOMEM, "slice workspace");
    if (hipHostMalloc((void**)&ws->h_active, sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
      return set_error(GW_ENOMEM, "slice pinned flag");
    if (hipMalloc((void**)&ws->dev, sizeof(SliceDev)) != hipSuccess) return set_error(GW_ENOMEM, "slice parameters");
  }
  if (ws->cap >= k) {
    *out = ws;
    return GW_OK;
  }
  if (ws->mem) (void)hipFree(ws->mem);
  ws->mem = nullptr;
  ws->cap = 0;
  // doubles: t_lo, t_hi, d[4], cand_t[2], cand[26], cand_logl[2]; ints: flags, n_out[2], n_shrink, n_evals,
  // slot_ok[2], then the active counter
  const size_t nd = (size_t)k * (1 + 1 + kMaxBlock + 2 + 26 + 2);
  const size_t ni = (size_t)k * (1 + 2 + 1 + 1 + 2) + 1;
  char* m = nullptr;
  gw_status s = check_hip(hipMalloc((void**)&m, nd * sizeof(double) + ni * sizeof(int32_t)), "slice workspace");
  if (s != GW_OK) return s;
  double* dp = (double*)m;
  ws->S.t_lo = dp; dp += k;
  ws->S.t_hi = dp; dp += k;
  ws->S.d = dp; dp += k * kMaxBlock;
  ws->S.cand_t = dp; dp += 2 * k;
  ws->cand = dp; dp += 26 * k;
  ws->cand_logl = dp; dp += 2 * k;
  int32_t* ip = (int32_t*)dp;
  ws->S.flags = ip; ip += k;
  ws->S.n_out = ip; ip += 2 * k;
  ws->S.n_shrink = ip; ip += k;
  ws->S.n_evals = ip; ip += k;
  ws->S.slot_ok = ip; ip += 2 * k;
  ws->S.n_active = ip;
  ws->mem = m;
  ws->cap = k;
  *out = ws;
  return GW_OK;
}

namespace gw {
void slice_free(gw_ctx* ctx) {
  gw_slice_ws* ws = ctx->slice;
  if (!ws) return;
  if (ws->exec) (void)hipGraphExecDestroy(ws->exec);
  if (ws->graph) (void)hipGraphDestroy(ws->graph);
  if (ws->cap_stream) (void)hipStreamDestroy(ws->cap_stream);
  if (ws->mem) (void)hipFree(ws->mem);
  if (ws->dev) (void)hipFree(ws->dev);
  if (ws->h_active) (void)hipHostFree(ws->h_active);
  delete ws;
  ctx->slice = nullptr;
}
}  // namespace gw
