// Constrained hit-and-run slice moves over k chains (Sec. II.C and III.B,
// Eq. block_cprior).  Each chain moves one Gibbs block of unit-cube
// coordinates along t -> x + t d with d = L u (u a random unit vector, L the
// Cholesky factor of the block covariance), stepping the bracket out while its
// ends satisfy log L > log L*, then shrinking it until a point inside the
// constraint is found; a sweep takes the blocks in order.  Chains advance in
// rounds: a propose kernel writes every chain's candidate points as parameter
// vectors, the batched likelihood evaluates them all, and an update kernel
// moves each chain's state machine (to its next block once one is done); the
// host checks for completion every few rounds.  With a prescreen network the
// round also runs the network on every candidate's unit-cube point between
// propose and likelihood: a candidate predicted below log L* - margin is taken
// as outside the constraint without a likelihood call, unless it is drawn for
// the audit; every accepted point has an exact log L.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "gw_ctx.h"
#include "gw_rng.h"

namespace gw {

constexpr int kSliceDim = 11;
constexpr int kMaxBlock = 11;   // coordinates per block (a block may hold all of them)
constexpr int kMaxBlocks = 16;  // blocks per sweep
constexpr int kCholPack = 160;  // doubles of packed Cholesky factors per sweep

// Uniforms before the shrink draws of a block of bd coordinates: one
// Box-Muller pair per two coordinates (at least two pairs), the bracket
// offset, then the split of the stepping-out budget between the two ends.
__host__ __device__ inline int uni_fixed(int bd) { return (bd <= 4 ? 4 : 2 * ((bd + 1) / 2)) + 2; }

// How the sampler's last coordinate is read: t_c (phase and distance
// marginalised) or d_L (phase and time marginalised).
struct CubeMap {
  int32_t time_marg;  // 0: coordinate 10 is t_c; 1: coordinate 10 is d_L
  double d3_lo, d3_span;  // d_L^3 at the lower end of its prior, and the range of d_L^3
  // Detector sky frame: coordinates 7 and 8 are the azimuth 2 pi u and the
  // zenith acos(1 - 2 u) about the baseline nb of two detectors (e1, e2
  // across it, Earth-fixed); with det_time, coordinate 10 is the arrival
  // time at the first detector (position ra_m, in m).
  int32_t sky, det_time;
  double nb[3], e1[3], e2[3], ra_m[3];
  double gmst;
};

// One sweep: every chain visits blocks b = 0 .. nb - 1 in order, block b with
// Philox counter (counter + b).  Chains are independent, so a chain starts its
// next block as soon as it finishes one; each chain's moves are exactly those
// of nb successive one-block steps.  A single slice_step is the nb = 1 case.
struct SweepParams {
  int32_t nb;
  int32_t bd[kMaxBlocks];
  int32_t block[kMaxBlocks][kMaxBlock];
  int32_t choff[kMaxBlocks];  // block b's lower factor: chol[choff[b] + i * bd + j]
  double chol[kCholPack];
  double w;
  double logl_star;
  int32_t max_out, max_shrink;
  uint64_t seed, counter;
  const double* uniforms;  // one-block calls: [k][uni_fixed(bd) + max_shrink], or null
  int64_t k;
  double* x;
  double* logl;
  // Full band: candidates go to the likelihood as row lists (lists = 1).
  // Waveform cache (cache = 1): block kinds 0 slow (changes the intrinsic
  // waveform), 1 extrinsic (sky and time: cached waveform, new delays),
  // 2 projection only (psi, iota: cached sums z_i).
  int32_t lists;
  int32_t cache;
  CubeMap cm;
  int32_t n_det;
  int32_t kind[kMaxBlocks];
  // prescreen: screen = 1 runs the network; a candidate needs its exact log L
  // when the prediction is >= cut (= log L* - margin) or when its audit draw
  // (Philox4x64-10, key (seed, 1), counter (counter + b, c, kind, index),
  // word 0, mapped to (0, 1)) is below audit_frac
  int32_t screen;
  double cut;
  double audit_frac;
  // record = 1 appends every exactly evaluated candidate (unit-cube point,
  // log L) to the ring buffer rec_x / rec_l at slot (*rec_count)++ mod rec_cap
  int32_t record;
  int64_t rec_cap;
  double* rec_x;
  double* rec_l;
  unsigned long long* rec_count;
};

// passed by value to the kernel that copies it to the device
static_assert(sizeof(SweepParams) <= 4096, "sweep parameters must fit a kernel argument block");
static_assert(GW_MAX_BLOCK == kMaxBlock, "block stride of the sweep arguments");

// Per-chain state (structure of arrays inside one device allocation).
struct SliceState {
  double* t_lo;
  double* t_hi;
  double* d;        // [k][kMaxBlock]
  double* cand_t;   // [k][2]
  int32_t* flags;   // [k]: bit0 lo stepping, bit1 hi stepping, bit2 sweep done
  int32_t* n_out;   // [k][2]: steps left to each end's share of the stepping-out budget
  int32_t* n_shrink;
  int32_t* n_evals;  // likelihood calls in the current block
  int32_t* slot_ok;  // [k][2]: candidate inside the cube and needs a likelihood
  int32_t* cur;      // current block
  int32_t* tot_evals;
  int32_t* n_caps;   // blocks whose shrink cap was hit
  int32_t* n_active;  // [2] chains still moving after a round (the fused rounds alternate)
  // row lists and waveform cache bookkeeping (list mode only)
  int32_t* rkind;      // [2k]: 0 no likelihood, 1 full, 2 cached waveform, 3 cached sums
  int32_t* zsrc;       // [2k]: slot whose cached sums the row uses, or -1
  int32_t* build_list;  // [k]: chains whose waveform is rebuilt after this round
  int32_t* build_src;  // [k]: the candidate row each rebuild takes its coefficients from
  int32_t* dirty;      // [k]: the chain's cached waveform is older than its point
  int32_t* slow_rows;  // [2k]
  int32_t* stream_rows;  // [2k]
  int32_t* counts;     // [3]: rows in the two lists, chains in build_list
  unsigned long long* kind_tot;  // [3]: evaluations by kind over the sweep
  double* zrow;        // [2k][2 n_det]: every row's sums z_i
  double* zc;          // [k][2 n_det]: the sums at each chain's current point, then
                       // [2k][2 n_det]: the cached-waveform rows' sums
  // prescreen
  double* ucand;       // [2k][11]: each slot's unit-cube point (the network's input)
  double* pred;        // [2k]: the network's log L
  int32_t* scr;        // [2k]: 0 evaluated (predicted inside), 1 screened out, 2 audited
  int32_t* side_tests; // [k][2]: stepping-out tests made at each end in this block
  unsigned long long* scr_tot;  // [3]: screened out, audited, audited and inside (false negatives)
};

// Uniform j of chain c in block b: explicit table, or Philox word j % 4 of
// counter (counter_base + b, c, j / 4, 0) under key (seed, 0), mapped to (0, 1).
__device__ inline double slice_uniform(const SweepParams& P, int b, int64_t c, int j) {
  if (P.uniforms) return P.uniforms[c * (uni_fixed(P.bd[b]) + P.max_shrink) + j];
  uint64_t ctr[4] = {P.counter + (uint64_t)b, (uint64_t)c, (uint64_t)(j >> 2), 0ull};
  philox4x64(ctr, P.seed, 0ull);
  return philox_unit(ctr[j & 3]);
}

// Audit draw of a screened candidate: test ``idx`` of kind ``kind`` (0 lower
// end, 1 upper end, 2 shrink draw) of chain c in block b.
__device__ inline double audit_uniform(const SweepParams& P, int b, int64_t c, int kind, int idx) {
  uint64_t ctr[4] = {P.counter + (uint64_t)b, (uint64_t)c, (uint64_t)kind, (uint64_t)idx};
  philox4x64(ctr, P.seed, 1ull);
  return philox_unit(ctr[0]);
}

// Unit cube -> 13-column parameter vector.  Coordinate 10 is t_c in [-0.1,
// 0.1] s (d_L = 1, phi_c = 0, both marginalised) or, with time_marg, d_L with
// a prior proportional to d_L^2 (inverse CDF (d3_lo + u d3_span)^(1/3); t_c =
// 0 and phi_c = 0 marginalised).
__device__ inline void prior_transform(const double* u, double* th, const CubeMap& cm) {
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
  if (cm.time_marg) {
    th[6] = cbrt(fma(u[10], cm.d3_span, cm.d3_lo));
    th[12] = 0.0;
  }
  if (cm.sky) {
    double sk, ck, sz, cz;
    sincos(kTwoPi * u[7], &sk, &ck);
    sincos(acos(1.0 - 2.0 * u[8]), &sz, &cz);
    double s[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) s[i] = cz * cm.nb[i] + sz * (ck * cm.e1[i] + sk * cm.e2[i]);
    th[9] = asin(fmin(1.0, fmax(-1.0, s[2])));
    double ra = atan2(s[1], s[0]) + cm.gmst;
    if (ra < 0.0) ra += kTwoPi;
    else if (ra >= kTwoPi) ra -= kTwoPi;
    th[8] = ra;
    if (cm.det_time && !cm.time_marg)
      th[12] = (-0.1 + 0.2 * u[10]) + (s[0] * cm.ra_m[0] + s[1] * cm.ra_m[1] + s[2] * cm.ra_m[2]) / kLightSpeed;
  }
}

// Start block b for chain c: direction d = L u (u from Box-Muller normals,
// pair p from uniforms 2p and 2p + 1, normalised), bracket [-r w, (1 - r) w]
// with r the uniform after the direction ones, and the stepping-out budget
// m = 2 max_out + 1 split by the next uniform V into J = floor(m V) steps for
// the lower end and m - 1 - J for the upper one (Neal 2003, Sec. 4.1: with
// the split drawn at random, every point of the final bracket is equally
// likely to have produced it, so the move stays reversible when a cap
// binds).  Returns the chain's new flags.
__device__ inline int start_block(const SweepParams& P, const SliceState& S, int64_t c, int b) {
  const int bd = P.bd[b];
  const int nfix = uni_fixed(bd);
  // the fixed uniforms 0 .. nfix - 1 (nfix <= 14): each Philox block of four
  // is drawn once, giving the values slice_uniform returns one at a time
  double un[16];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (4 * q < nfix) {
      if (P.uniforms) {
#pragma unroll
        for (int w = 0; w < 4; ++w)
          un[4 * q + w] = 4 * q + w < nfix ? P.uniforms[c * (nfix + P.max_shrink) + 4 * q + w] : 0.5;
      } else {
        uint64_t ctr[4] = {P.counter + (uint64_t)b, (uint64_t)c, (uint64_t)q, 0ull};
        philox4x64(ctr, P.seed, 0ull);
#pragma unroll
        for (int w = 0; w < 4; ++w) un[4 * q + w] = philox_unit(ctr[w]);
      }
    } else {
#pragma unroll
      for (int w = 0; w < 4; ++w) un[4 * q + w] = 0.5;
    }
  }
  // normals for the block's coordinates only
  double z[kMaxBlock + 1];
#pragma unroll
  for (int p = 0; p < (kMaxBlock + 1) / 2; ++p) {
    z[2 * p] = z[2 * p + 1] = 0.0;
    if (2 * p < bd) {
      const double r = sqrt(-2.0 * log(un[2 * p]));
      double sn, cs;
      sincos(kTwoPi * un[2 * p + 1], &sn, &cs);
      z[2 * p] = r * cs;
      z[2 * p + 1] = r * sn;
    }
  }
  double nrm = 0.0;
#pragma unroll
  for (int j = 0; j < kMaxBlock; ++j)
    if (j < bd) nrm += z[j] * z[j];
  nrm = sqrt(nrm);
  const double* L = P.chol + P.choff[b];
  for (int a = 0; a < kMaxBlock; ++a) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxBlock; ++q)
      if (q < bd && a < bd) v += L[a * bd + q] * (z[q] / nrm);
    S.d[c * kMaxBlock + a] = a < bd ? v : 0.0;
  }
  double off = 0.0, vsplit = 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    if (j == nfix - 2) off = un[j];
    if (j == nfix - 1) vsplit = un[j];
  }
  S.t_lo[c] = -off * P.w;
  S.t_hi[c] = (1.0 - off) * P.w;
  const int budget = 2 * P.max_out + 1;
  const int j_lo = (int)floor((double)budget * vsplit);
  const int j_hi = budget - 1 - j_lo;
  S.n_out[2 * c] = j_lo;
  S.n_out[2 * c + 1] = j_hi;
  S.side_tests[2 * c] = 0;
  S.side_tests[2 * c + 1] = 0;
  S.n_shrink[c] = 0;
  S.n_evals[c] = 0;
  S.cur[c] = b;
  return (j_lo > 0 ? 1 : 0) | (j_hi > 0 ? 2 : 0);
}

// The current block of chain c ends (moved, or kept when capped): count it
// and start the next block, or mark the sweep done.  Returns the new flags.
__device__ inline int finish_block(const SweepParams& P, const SliceState& S, int64_t c, bool capped) {
  S.tot_evals[c] += S.n_evals[c];
  if (capped) S.n_caps[c] += 1;
  const int b = S.cur[c] + 1;
  return b < P.nb ? start_block(P, S, c, b) : 4;
}

__device__ inline bool make_point(const SweepParams& P, int b, const SliceState& S, const double* x0, int64_t c,
                                  double t, double* u) {
  for (int j = 0; j < kSliceDim; ++j) u[j] = x0[c * kSliceDim + j];
  bool inside = true;
  for (int a = 0; a < P.bd[b]; ++a) {
    const int j = P.block[b][a];
    const double v = x0[c * kSliceDim + j] + t * S.d[c * kMaxBlock + a];
    inside = inside && v >= 0.0 && v <= 1.0;
    u[j] = v;
  }
  return inside;
}

__global__ void k_sweep_set(SweepParams* D, SweepParams P, unsigned long long* kind_tot,
                            unsigned long long* scr_tot) {
  *D = P;
  for (int i = 0; i < 3; ++i) {
    kind_tot[i] = 0;
    scr_tot[i] = 0;
  }
}

// Threads per workgroup of the sweep kernels (one per chain): the bound lets
// the chain's state (a point, a direction, the block's Cholesky row) stay in
// registers instead of scratch memory.
constexpr int kSweepThreads = 256;

__global__ void __launch_bounds__(kSweepThreads) k_sweep_init(const SweepParams* __restrict__ D, SliceState S) {
  const SweepParams& P = *D;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.k) return;
  S.tot_evals[c] = 0;
  S.n_caps[c] = 0;
  S.flags[c] = start_block(P, S, c, 0);
}

// Write the candidates of every chain that is still moving: the two bracket
// ends while stepping out, else one shrink draw (points outside the cube
// count as rejections immediately, without a likelihood call).
__device__ inline void propose_chain(const SweepParams& P, const SliceState& S, double* __restrict__ cand,
                                     int64_t c) {
  const double* __restrict__ x0 = P.x;
  int fl = S.flags[c];
  double u[kSliceDim];
  int ok[2] = {0, 0};
  // a block whose shrink draws all leave the cube ends here without a call;
  // the next block (if any) then proposes in the same round
  for (int guard = 0; guard <= kMaxBlocks && !(fl & 4) && !ok[0] && !ok[1]; ++guard) {
    const int b = S.cur[c];
    if (fl & 3) {
      #pragma unroll
      for (int side = 0; side < 2; ++side) {
        if (!(fl & (1 << side))) continue;
        const double t = side == 0 ? S.t_lo[c] : S.t_hi[c];
        if (make_point(P, b, S, x0, c, t, u)) {
          prior_transform(u, cand + (2 * c + side) * 13, P.cm);
          S.cand_t[2 * c + side] = t;
          ok[side] = 1;
          if (P.screen || P.record)
            for (int j = 0; j < kSliceDim; ++j) S.ucand[(2 * c + side) * kSliceDim + j] = u[j];
          if (P.screen)
            S.scr[2 * c + side] =
                audit_uniform(P, b, c, side, S.side_tests[2 * c + side]) < P.audit_frac ? 2 : 0;
        } else {
          fl &= ~(1 << side);  // outside the cube: this side stops here
        }
      }
    }
    if (!(fl & 3)) {
      // shrinking: draw until a point lies in the cube (no likelihood needed
      // for the others) or the cap is reached
      while (S.n_shrink[c] < P.max_shrink) {
        const double v = slice_uniform(P, b, c, uni_fixed(P.bd[b]) + S.n_shrink[c]);
        const double t = S.t_lo[c] + v * (S.t_hi[c] - S.t_lo[c]);
        if (make_point(P, b, S, x0, c, t, u)) {
          prior_transform(u, cand + 2 * c * 13, P.cm);
          S.cand_t[2 * c] = t;
          ok[0] = 1;
          if (P.screen || P.record)
            for (int j = 0; j < kSliceDim; ++j) S.ucand[2 * c * kSliceDim + j] = u[j];
          if (P.screen) S.scr[2 * c] = audit_uniform(P, b, c, 2, S.n_shrink[c]) < P.audit_frac ? 2 : 0;
          break;
        }
        if (t < 0.0) S.t_lo[c] = t;
        else S.t_hi[c] = t;
        S.n_shrink[c] += 1;
      }
      if (!ok[0]) fl = finish_block(P, S, c, true);  // cap reached: keep the point
    }
  }
  // rows that need no likelihood get an unphysical vector (cheap -inf)
  #pragma unroll
  for (int side = 0; side < 2; ++side)
    if (!ok[side]) {
      double* th = cand + (2 * c + side) * 13;
      for (int j = 0; j < 13; ++j) th[j] = 0.0;
      th[1] = -1.0;
      if (P.screen) {
        for (int j = 0; j < kSliceDim; ++j) S.ucand[(2 * c + side) * kSliceDim + j] = 0.5;
        S.scr[2 * c + side] = 0;
      }
    }
  S.slot_ok[2 * c] = ok[0];
  S.slot_ok[2 * c + 1] = ok[1];
  S.flags[c] = fl;
  if (P.lists) {
    // an extrinsic block whose cached waveform is stale evaluates in full
    // (for one round, until the rebuild queued below has run)
    int kd = 0;
    if (!(fl & 4)) {
      const int kb = P.cache ? P.kind[S.cur[c]] : 0;
      kd = kb == 1 && S.dirty[c] ? 1 : 1 + kb;
    }
    S.rkind[2 * c] = ok[0] ? kd : 0;
    S.rkind[2 * c + 1] = ok[1] ? kd : 0;
  }
}

__global__ void __launch_bounds__(kSweepThreads) k_sweep_propose(const SweepParams* __restrict__ D, SliceState S, double* __restrict__ cand) {
  const SweepParams& P = *D;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) *S.n_active = 0;
  if (c >= P.k) return;
  propose_chain(P, S, cand, c);
}

// Prescreen decision per candidate slot (after the network has written pred):
// a slot predicted below the cut and not audited gets no likelihood call.
__global__ void k_sweep_screen(const SweepParams* __restrict__ D, SliceState S, double* __restrict__ cand) {
  const SweepParams& P = *D;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 2 * P.k || !S.slot_ok[r]) return;
  if (S.pred[r] >= P.cut) {
    S.scr[r] = 0;
    return;
  }
  if (S.scr[r] == 2) return;  // audited: evaluated although predicted outside
  S.scr[r] = 1;
  if (P.lists) S.rkind[r] = 0;
  double* th = cand + r * 13;  // the batched forms: a row that costs an unphysical -inf
  for (int j = 0; j < 13; ++j) th[j] = 0.0;
  th[1] = -1.0;
}

// Append an exactly evaluated candidate to the caller's ring buffer.
__device__ inline void record_pair(const SweepParams& P, const SliceState& S, int64_t slot, double v) {
  if (!P.record) return;
  const int64_t pos = (int64_t)(atomicAdd(P.rec_count, 1ull) % (unsigned long long)P.rec_cap);
  for (int j = 0; j < kSliceDim; ++j) P.rec_x[pos * kSliceDim + j] = S.ucand[slot * kSliceDim + j];
  P.rec_l[pos] = v;
}

// Returns the chain's flags (4 set once its sweep is done, also when it was
// done before this round).
__device__ inline int update_chain(const SweepParams& P, const SliceState& S, const double* __restrict__ cand_logl,
                                   int64_t c) {
  double* __restrict__ x = P.x;
  double* __restrict__ logl = P.logl;
  int fl = S.flags[c];
  if (fl & 4) return fl;
  const int b = S.cur[c];  // the block of this round's rows
  const bool stepping = (fl & 3) != 0;
  bool moved = false;
  if (stepping) {
    for (int side = 0; side < 2; ++side) {
      if (!S.slot_ok[2 * c + side]) continue;
      S.side_tests[2 * c + side] += 1;
      bool in;
      if (P.screen && S.scr[2 * c + side] == 1) {
        atomicAdd(&S.scr_tot[0], 1ull);
        in = false;
      } else {
        S.n_evals[c] += 1;
        in = cand_logl[2 * c + side] > P.logl_star;
        record_pair(P, S, 2 * c + side, cand_logl[2 * c + side]);
        if (P.screen && S.scr[2 * c + side] == 2) {
          atomicAdd(&S.scr_tot[1], 1ull);
          if (in) atomicAdd(&S.scr_tot[2], 1ull);
        }
      }
      int left = S.n_out[2 * c + side];  // > 0 while this end is active
      if (in && left > 0) {
        if (side == 0) S.t_lo[c] -= P.w;
        else S.t_hi[c] += P.w;
        left -= 1;
        S.n_out[2 * c + side] = left;
        if (left == 0) fl &= ~(1 << side);
      } else {
        fl &= ~(1 << side);
      }
    }
  } else if (S.slot_ok[2 * c]) {
    double v = -INFINITY;
    if (P.screen && S.scr[2 * c] == 1) {
      atomicAdd(&S.scr_tot[0], 1ull);
    } else {
      S.n_evals[c] += 1;
      v = cand_logl[2 * c];
      record_pair(P, S, 2 * c, v);
      if (P.screen && S.scr[2 * c] == 2) {
        atomicAdd(&S.scr_tot[1], 1ull);
        if (v > P.logl_star) atomicAdd(&S.scr_tot[2], 1ull);
      }
    }
    const double t = S.cand_t[2 * c];
    if (v > P.logl_star) {
      for (int a = 0; a < P.bd[b]; ++a) {
        const int j = P.block[b][a];
        x[c * kSliceDim + j] += t * S.d[c * kMaxBlock + a];
      }
      logl[c] = v;
      if (P.cache) {
        // the chain's cached sums follow its point; a slow move also needs
        // the waveform rebuilt (from this row's coefficients)
        for (int j = 0; j < 2 * kMaxDet; ++j)
          if (j < 2 * P.n_det) S.zc[c * 2 * P.n_det + j] = S.zrow[2 * c * 2 * P.n_det + j];
        if (P.kind[b] == 0) S.dirty[c] = 1;
      }
      moved = true;
      fl = finish_block(P, S, c, false);
    } else {
      if (t < 0.0) S.t_lo[c] = t;
      else S.t_hi[c] = t;
      S.n_shrink[c] += 1;
      if (S.n_shrink[c] >= P.max_shrink) fl = finish_block(P, S, c, true);
    }
  }
  S.flags[c] = fl;
  if (!(fl & 4)) {
    // The waveform is rebuilt lazily, when a chain is in an extrinsic block
    // with a stale cache, after this round, from the coefficients of a row of
    // this round that has the chain's intrinsic parameters: the accepted row
    // after a move, else a row proposed in a block that keeps them (extrinsic
    // or projection-only) and not screened out.  A round without one (a slow
    // block ended at its shrink cap, an end that was never proposed) leaves
    // the cache stale; the next round's rows then evaluate in full and serve.
    if (P.cache && P.kind[S.cur[c]] == 1 && S.dirty[c]) {
      int src = -1;
      if (moved) {
        src = (int)(2 * c);
      } else if (P.kind[b] != 0) {
        for (int side = 1; side >= 0; --side) {
          const int64_t r = 2 * c + side;
          if (S.slot_ok[r] && !(P.screen && S.scr[r] == 1)) src = (int)r;
        }
      }
      if (src >= 0) {
        S.dirty[c] = 0;
        const int pos = atomicAdd(&S.counts[2], 1);
        S.build_list[pos] = (int32_t)c;
        S.build_src[pos] = src;
      }
    }
  }
  return fl;
}

// Count the chains still moving (flags without 4): one atomic per wave.
__device__ inline void count_active(int32_t* n_active, int fl) {
  const unsigned long long act = __ballot(!(fl & 4));
  if (act && (int)__lane_id() == __ffsll((long long)act) - 1) atomicAdd(n_active, (int32_t)__popcll(act));
}

__global__ void __launch_bounds__(kSweepThreads) k_sweep_update(const SweepParams* __restrict__ D, SliceState S, const double* __restrict__ cand_logl) {
  const SweepParams& P = *D;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.k) return;
  count_active(S.n_active, update_chain(P, S, cand_logl, c));
}

// One round's update followed by the next round's proposals, for calls with
// no waveform cache, prescreen or record: the same per-chain steps in the same
// order as k_sweep_update then k_sweep_propose, in one launch.  Moving chains
// are counted in n_active[slot]; n_active[slot ^ 1], which the next round
// counts into, is cleared here.
__global__ void __launch_bounds__(kSweepThreads) k_sweep_step(const SweepParams* __restrict__ D, SliceState S, const double* __restrict__ cand_logl, double* __restrict__ cand, int slot) {
  const SweepParams& P = *D;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) S.n_active[slot ^ 1] = 0;
  if (c >= P.k) return;
  count_active(S.n_active + slot, update_chain(P, S, cand_logl, c));
  propose_chain(P, S, cand, c);
}

// Row lists of the cached likelihood: rows of kind 1 and 2 in ascending
// order (one workgroup of 1024 threads), and each row's cached-sums slot.
__global__ void __launch_bounds__(1024) k_sweep_lists(const SweepParams* __restrict__ D, SliceState S) {
  __shared__ int32_t tot[2][16];
  const int64_t n = 2 * D->k;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  int32_t base0 = 0, base1 = 0;
  for (int64_t r0 = 0; r0 < n; r0 += 1024) {
    const int64_t r = r0 + threadIdx.x;
    const int kd = r < n ? S.rkind[r] : 0;
    if (r < n) S.zsrc[r] = kd == 3 ? (int32_t)(r >> 1) : -1;  // cached-waveform rows sum their partials
    const uint64_t m1 = __ballot(kd == 1), m2 = __ballot(kd == 2);
    if (lane == 0) {
      tot[0][wave] = __popcll(m1);
      tot[1][wave] = __popcll(m2);
    }
    __syncthreads();
    int32_t o0 = base0, o1 = base1, t0 = 0, t1 = 0;
    for (int w = 0; w < 16; ++w) {
      if (w < wave) {
        o0 += tot[0][w];
        o1 += tot[1][w];
      }
      t0 += tot[0][w];
      t1 += tot[1][w];
    }
    if (kd == 1) S.slow_rows[o0 + __popcll(m1 & below)] = (int32_t)r;
    if (kd == 2) S.stream_rows[o1 + __popcll(m2 & below)] = (int32_t)r;
    base0 += t0;
    base1 += t1;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    S.counts[0] = base0;
    S.counts[1] = base1;
    S.counts[2] = 0;  // the update kernel appends the chains to rebuild
  }
  // cached-sums rows, for the per-kind totals
  int32_t n3 = 0;
  for (int64_t r = threadIdx.x; r < n; r += 1024) n3 += S.rkind[r] == 3;
  for (int off = 32; off > 0; off >>= 1) n3 += __shfl_xor(n3, off);
  if (lane == 0) tot[0][wave] = n3;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t3 = 0;
    for (int w = 0; w < 16; ++w) t3 += tot[0][w];
    S.kind_tot[0] += (unsigned long long)base0;
    S.kind_tot[1] += (unsigned long long)base1;
    S.kind_tot[2] += (unsigned long long)t3;
  }
}

// Cache set-up at the start of a sweep: row 2c evaluates chain c's current
// point in full (row 2c + 1 needs nothing) ...
__global__ void k_cache_init0(const SweepParams* __restrict__ D, SliceState S, double* __restrict__ cand) {
  const SweepParams& P = *D;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.k) return;
  prior_transform(P.x + c * kSliceDim, cand + 2 * c * 13, P.cm);
  double* th = cand + (2 * c + 1) * 13;
  for (int j = 0; j < 13; ++j) th[j] = 0.0;
  th[1] = -1.0;
  S.rkind[2 * c] = 1;
  S.rkind[2 * c + 1] = 0;
}

// ... and its sums seed the chain's cached sums; its waveform is built when
// first needed.
__global__ void k_cache_init1(const SweepParams* __restrict__ D, SliceState S) {
  const SweepParams& P = *D;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.k) return;
  for (int j = 0; j < 2 * P.n_det; ++j) S.zc[c * 2 * P.n_det + j] = S.zrow[2 * c * 2 * P.n_det + j];
  S.dirty[c] = 1;
}

__global__ void k_prior_transform(const double* __restrict__ x, int64_t n, CubeMap cm, double* __restrict__ theta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) prior_transform(x + i * kSliceDim, theta + i * 13, cm);
}

__global__ void k_sweep_finish(const SweepParams* __restrict__ D, SliceState S, int32_t* n_evals, int32_t* status) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= D->k) return;
  if (n_evals) n_evals[c] = S.tot_evals[c];
  if (status) status[c] = S.n_caps[c];
}

}  // namespace gw

using namespace gw;

// What a captured round group bakes in: any change means a new capture.
struct SliceGraphKey {
  int64_t k;
  int32_t like, marg, prec, cache;
  const void *ws_mem, *coef, *partial, *zbuf, *het, *wc, *mlp;
  uint64_t mlp_scale, gen;
  const void *tm_mom, *tm_ccoef, *tm_basis, *tm_tab, *tm_idx;
  int32_t het_wpb, het_grid, het_ech, full_tpb, full_chunks, full_kernel;
  int32_t tm_nch, tm_nslot, tm_nsplit, fused, pinned, pad;
  bool operator==(const SliceGraphKey& o) const { return memcmp(this, &o, sizeof(*this)) == 0; }
};

struct gw_slice_ws {
  int64_t cap = 0;
  void* mem = nullptr;
  double* cand = nullptr;       // [2k][13]
  double* cand_logl = nullptr;  // [2k]
  int32_t* h_active = nullptr;  // pinned host [2]: chains still moving after a group, double-buffered
  unsigned long long* h_kinds = nullptr;  // pinned host [6]: evaluation kinds, then prescreen counts
  hipEvent_t ev[2] = {nullptr, nullptr};  // readback of h_active[i] complete
  SliceState S{};
  SweepParams* dev = nullptr;   // device parameter block
  float2* wc = nullptr;         // waveform cache (block moments) [cap_wc][slot_f2]
  int64_t cap_wc = 0;
  int64_t slot_f2 = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  SliceGraphKey key{};
  bool have_graph = false;
};

static gw_status slice_ws(gw_ctx* ctx, int64_t k, gw_slice_ws** out);
static gw_status slice_wcache(gw_ctx* ctx, gw_slice_ws* ws, int64_t k);

struct SweepCall {
  int32_t like, marg, prec, use_graph;
  int32_t* n_evals;
  int32_t* status;
  int32_t cache;
  int64_t* eval_kinds;  // host [3] or null
  int32_t lists;        // full band: row-list likelihood (always with the cache)
  gw_mlp* mlp;          // prescreen network or null
  int64_t* screen_stats;  // host [3] or null
};

// Launch shape of the row-list likelihood: 64 rows per workgroup, its four
// waves splitting chunks of about 512 bins (the rows of a round are few, so
// the bins supply the parallelism).
void gw::cached_shape(const gw_ctx* ctx, int* tpb, int* nch) {
  int64_t c = (ctx->geom.n_freq + 511) / 512;
  c = (c + 7) / 8 * 8;
  *tpb = 256;
  *nch = (int)c;
}

gw_status gw::cached_reserve(gw_ctx* ctx, int64_t n) {
  int tpb, nch;
  cached_shape(ctx, &tpb, &nch);
  gw_status s = ensure_buffer(&ctx->coef, &ctx->coef_cap, (int64_t)C_NCOEF * n, "coefficient workspace");
  if (s == GW_OK) s = ensure_buffer(&ctx->partial, &ctx->partial_cap, (int64_t)nch * 2 * ctx->n_det * n, "partials");
  if (s == GW_OK) s = ensure_buffer(&ctx->zbuf, &ctx->zbuf_cap, 2 * n, "marginal workspace");
  return s;
}

// Likelihood of the round's 2k candidate rows into ws->cand_logl.
static gw_status eval_rows(gw_ctx* ctx, gw_slice_ws* ws, int64_t k, const SweepCall& a, hipStream_t st) {
  const int64_t n = 2 * k;
  if (!a.lists) return loglike_batch(ctx, ws->cand, n, a.like, a.marg, a.prec, ws->cand_logl, st);
  gw_status s = cached_reserve(ctx, n);
  if (s != GW_OK) return s;
  int tpb, nch;
  cached_shape(ctx, &tpb, &nch);
  hipLaunchKernelGGL(k_sweep_lists, dim3(1), dim3(1024), 0, st, (const SweepParams*)ws->dev, ws->S);
  s = check_hip(hipGetLastError(), "row list launch");
  if (s == GW_OK) s = launch_prologue(ctx, ws->cand, n, a.marg, ctx->coef, n, st);
  if (s == GW_OK)
    s = launch_cached(ctx, ctx->coef, n, a.prec, tpb, nch, ws->S.slow_rows, ws->S.stream_rows, ws->S.counts, 2,
                      nullptr, a.cache ? ws->wc : nullptr, nullptr, ctx->partial, st);
  if (s == GW_OK)
    s = launch_epilogue_cached(ctx, ctx->partial, nch, ctx->coef, n, n, a.marg, a.prec, ws->cand_logl, ws->S.zsrc,
                               ws->S.zc, ws->S.zrow, st);
  return s;
}

// Capture one round group into a graph (re-captured when anything it bakes in
// changes) on the workspace's own capture stream.  Buffers the likelihood
// would grow are reserved first: no allocation may happen during capture.
template <class Group>
static gw_status slice_graph(gw_ctx* ctx, gw_slice_ws* ws, int64_t k, const SweepCall& a, bool fused, bool pinned,
                             Group group) {
  const int64_t n = 2 * k;
  gw_status s = a.lists ? cached_reserve(ctx, n) : a.like == GW_HET ? het_reserve(ctx, n) : full_reserve(ctx, n);
  if (s == GW_OK && a.marg == GW_MARG_PHASE_TIME) s = tmarg_reserve(ctx, n, a.like);
  if (s != GW_OK) return s;
  SliceGraphKey key;
  memset(&key, 0, sizeof(key));
  key.k = k;
  key.like = a.like;
  key.marg = a.marg;
  key.prec = a.prec;
  key.cache = a.cache + 2 * a.lists;
  key.wc = ws->wc;
  key.ws_mem = ws->mem;
  key.coef = ctx->coef;
  key.partial = ctx->partial;
  key.zbuf = ctx->zbuf;
  key.het = ctx->het;
  het_shape_key(ctx, &key.het_wpb, &key.het_grid, &key.het_ech);
  key.full_tpb = ctx->full_tpb;
  key.full_chunks = ctx->full_chunks;
  key.full_kernel = ctx->full_kernel;
  key.mlp = a.mlp;
  key.mlp_scale = a.mlp ? mlp_scale_version(a.mlp) : 0;
  key.gen = ctx->gen;
  key.fused = fused ? 1 : 0;
  key.pinned = pinned ? 1 : 0;
  if (a.marg == GW_MARG_PHASE_TIME) {
    key.tm_mom = ctx->tm_mom;
    key.tm_ccoef = ctx->tm_ccoef;
    key.tm_basis = ctx->tm_basis;
    het_tm_key(ctx, &key.tm_tab, &key.tm_idx, &key.tm_nch, &key.tm_nslot, &key.tm_nsplit);
  }
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

// The cube map for a marginalisation mode: with the time marginal, d_L spans
// the context's distance grid (prior proportional to d_L^2).
static gw_status cube_map(const gw_ctx* ctx, int32_t marg, CubeMap* cm) {
  *cm = CubeMap{};
  if (ctx->sky_frame) {
    // baseline n = (r_b - r_a) / |r_b - r_a|; e1 = z made orthogonal to n (x
    // when n is nearly along z); e2 = n x e1
    const double* ra = ctx->geom.pos[ctx->sky_a];
    const double* rb = ctx->geom.pos[ctx->sky_b];
    double n[3] = {rb[0] - ra[0], rb[1] - ra[1], rb[2] - ra[2]};
    const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (double& v : n) v /= nn;
    double ref[3] = {0.0, 0.0, 1.0};
    if (fabs(n[2]) > 0.99) {
      ref[0] = 1.0;
      ref[2] = 0.0;
    }
    const double rn = ref[0] * n[0] + ref[1] * n[1] + ref[2] * n[2];
    double e1[3] = {ref[0] - rn * n[0], ref[1] - rn * n[1], ref[2] - rn * n[2]};
    const double ne = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (double& v : e1) v /= ne;
    const double e2[3] = {n[1] * e1[2] - n[2] * e1[1], n[2] * e1[0] - n[0] * e1[2], n[0] * e1[1] - n[1] * e1[0]};
    cm->sky = 1;
    cm->det_time = ctx->sky_det_time;
    for (int i = 0; i < 3; ++i) {
      cm->nb[i] = n[i];
      cm->e1[i] = e1[i];
      cm->e2[i] = e2[i];
      cm->ra_m[i] = ra[i];
    }
    cm->gmst = ctx->geom.gmst;
  }
  if (marg != GW_MARG_PHASE_TIME) return GW_OK;
  if (ctx->h_dist_grid.size() < 2) return set_error(GW_ESTATE, "time-marginal sampler needs a distance grid");
  const double lo = ctx->h_dist_grid.front(), hi = ctx->h_dist_grid.back();
  cm->time_marg = 1;
  cm->d3_lo = lo * lo * lo;
  cm->d3_span = hi * hi * hi - cm->d3_lo;
  return GW_OK;
}

// Validation shared by both entry points.
static gw_status check_sweep(const char* who, int64_t k, const double* x, const double* logl, double w,
                             int32_t max_out, int32_t max_shrink, int32_t like, int32_t marg, const gw_ctx* ctx) {
  if (k < 0) return set_error(GW_EINVAL, "%s: k < 0", who);
  if (k > 0 && (!x || !logl)) return set_error(GW_EINVAL, "%s: null pointer", who);
  if (!(w > 0.0) || !isfinite(w)) return set_error(GW_EINVAL, "%s: w must be > 0", who);
  if (max_out < 0 || max_out > 10000 || max_shrink < 1 || max_shrink > 10000)
    return set_error(GW_EINVAL, "%s: max_out 0..10000, max_shrink 1..10000", who);
  if (marg == GW_MARG_NONE)
    return set_error(GW_ENOTSUP, "%s: the 11-D sampler needs phi_c and d_L, or phi_c and t_c, marginalised", who);
  if (marg != GW_MARG_PHASE_DIST && marg != GW_MARG_PHASE_TIME)
    return set_error(GW_ENOTSUP, "%s: marg must be GW_MARG_PHASE_DIST or GW_MARG_PHASE_TIME", who);
  if (like != GW_FULL && like != GW_HET)
    return set_error(GW_EINVAL, "%s: like must be GW_FULL or GW_HET", who);
  if (like == GW_HET && !ctx->het)
    return set_error(GW_ESTATE, "%s: heterodyne_setup has not been called", who);
  return GW_OK;
}

// Prescreen arguments shared by both entry points.
static gw_status set_screen(const char* who, const gw_ctx* ctx, gw_mlp* mlp, double margin, double audit_frac,
                            SweepParams& P) {
  P.screen = 0;
  if (!mlp) return GW_OK;
  if (mlp_ctx(mlp) != ctx) return set_error(GW_EINVAL, "%s: the prescreen network belongs to another context", who);
  if (!isfinite(margin)) return set_error(GW_EINVAL, "%s: margin must be finite", who);
  if (!(audit_frac >= 0.0 && audit_frac <= 1.0)) return set_error(GW_EINVAL, "%s: audit_frac in [0, 1]", who);
  P.screen = 1;
  P.cut = P.logl_star - margin;
  P.audit_frac = audit_frac;
  return GW_OK;
}

// Candidate recording arguments shared by both entry points.
static gw_status set_record(const char* who, double* rec_x, double* rec_logl, int64_t rec_cap,
                            unsigned long long* rec_count, SweepParams& P) {
  P.record = 0;
  if (!rec_x && !rec_logl && !rec_count) return GW_OK;
  if (!rec_x || !rec_logl || !rec_count || rec_cap < 1)
    return set_error(GW_EINVAL, "%s: rec_x, rec_logl and rec_count with rec_cap >= 1, or none of them", who);
  P.record = 1;
  P.rec_cap = rec_cap;
  P.rec_x = rec_x;
  P.rec_l = rec_logl;
  P.rec_count = rec_count;
  return GW_OK;
}

// Check one block (indices distinct in 0..10, 1..11 of them) and pack its
// lower Cholesky factor (row-major, stride ``ld``) into P.chol.  A block equal
// to an earlier one of the sweep (same coordinates and factor) shares its
// packed factor, so that one large block can be repeated.
static gw_status set_block(const char* who, SweepParams& P, int b, const int32_t* idx, int32_t bd, const double* L,
                           int ld, int* used) {
  if (bd < 1 || bd > kMaxBlock)
    return set_error(GW_EINVAL, "%s: block %d: block_dim 1..11", who, b);
  for (int i = 0; i < bd; ++i) {
    if (idx[i] < 0 || idx[i] >= kSliceDim)
      return set_error(GW_EINVAL, "%s: block %d: index 0..10", who, b);
    for (int j = 0; j < i; ++j)
      if (idx[j] == idx[i])
        return set_error(GW_EINVAL, "%s: block %d: repeated index", who, b);
  }
  P.bd[b] = bd;
  for (int i = 0; i < kMaxBlock; ++i) P.block[b][i] = i < bd ? idx[i] : 0;
  double f[kMaxBlock * kMaxBlock];
  for (int i = 0; i < bd; ++i)
    for (int j = 0; j < bd; ++j) f[i * bd + j] = j <= i ? L[i * ld + j] : 0.0;
  for (int c = 0; c < b; ++c) {
    if (P.bd[c] != bd) continue;
    bool same = true;
    for (int i = 0; i < bd && same; ++i) same = P.block[c][i] == idx[i];
    for (int i = 0; i < bd * bd && same; ++i) same = P.chol[P.choff[c] + i] == f[i];
    if (same) {
      P.choff[b] = P.choff[c];
      return GW_OK;
    }
  }
  if (*used + bd * bd > kCholPack)
    return set_error(GW_EINVAL, "%s: the distinct blocks' Cholesky factors exceed %d values", who, kCholPack);
  P.choff[b] = *used;
  for (int i = 0; i < bd * bd; ++i) P.chol[*used + i] = f[i];
  *used += bd * bd;
  return GW_OK;
}

// Run one sweep of P.nb blocks for all chains to completion.
static gw_status run_sweep(gw_ctx* ctx, const SweepParams& P, const SweepCall& a, hipStream_t st) {
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  gw_slice_ws* ws = nullptr;
  s = slice_ws(ctx, P.k, &ws);
  if (s == GW_OK && a.cache) s = slice_wcache(ctx, ws, P.k);
  if (s != GW_OK) return s;
  const int64_t k = P.k;
  const int tpb = kSweepThreads;
  const unsigned blocks = (unsigned)((k + tpb - 1) / tpb);
  if (a.mlp) {
    s = mlp_prepare(a.mlp, st);  // BF16 weights current before any capture or launch
    if (s != GW_OK) return s;
  }
  hipLaunchKernelGGL(k_sweep_set, dim3(1), dim3(1), 0, st, ws->dev, P, ws->S.kind_tot, ws->S.scr_tot);
  hipLaunchKernelGGL(k_sweep_init, dim3(blocks), dim3(tpb), 0, st, (const SweepParams*)ws->dev, ws->S);
  s = check_hip(hipGetLastError(), "slice init launch");
  if (s == GW_OK && a.cache) {
    // seed every chain's cached sums from a full evaluation of its current point
    hipLaunchKernelGGL(k_cache_init0, dim3(blocks), dim3(tpb), 0, st, (const SweepParams*)ws->dev, ws->S, ws->cand);
    s = check_hip(hipGetLastError(), "cache init launch");
    if (s == GW_OK) s = eval_rows(ctx, ws, k, a, st);
    if (s == GW_OK) {
      hipLaunchKernelGGL(k_cache_init1, dim3(blocks), dim3(tpb), 0, st, (const SweepParams*)ws->dev, ws->S);
      s = check_hip(hipGetLastError(), "cache init launch");
    }
  }
  // One group = 4 rounds of (propose, batched likelihood, update); after a
  // group the number of chains still moving is copied back.  A block takes at
  // most 2 max_out stepping rounds (both ends in parallel, their shares
  // summing to 2 max_out) and max_shrink shrink rounds, so after max_rounds
  // every chain is done.  Rounds after every
  // chain is done change nothing, so the next group is queued before the
  // previous group's count is read: the host waits on group g while group
  // g + 1 runs, and at most one group of idle rounds follows the last move.
  const int max_rounds = P.nb * (2 * P.max_out + 1 + P.max_shrink + 1);
  // Without a cache, prescreen or record, a round's update and the next
  // round's proposals run as one kernel (k_sweep_step) and the first
  // proposals are launched once before the groups.
  const bool fused = !a.cache && !a.mlp && !P.record;
  if (s == GW_OK && fused) {
    hipLaunchKernelGGL(k_sweep_propose, dim3(blocks), dim3(tpb), 0, st, (const SweepParams*)ws->dev, ws->S,
                       ws->cand);
    s = check_hip(hipGetLastError(), "slice propose launch");
  }
  auto group = [&](hipStream_t gs) -> gw_status {
    gw_status g = GW_OK;
    for (int r = 0; r < 4 && g == GW_OK; ++r) {
      if (!fused) {
        hipLaunchKernelGGL(k_sweep_propose, dim3(blocks), dim3(tpb), 0, gs, (const SweepParams*)ws->dev, ws->S,
                           ws->cand);
        g = check_hip(hipGetLastError(), "slice propose launch");
      }
      if (g == GW_OK && a.mlp) {
        g = mlp_infer(a.mlp, ws->S.ucand, 2 * k, ws->S.pred, gs);
        if (g == GW_OK) {
          hipLaunchKernelGGL(k_sweep_screen, dim3((unsigned)((2 * k + tpb - 1) / tpb)), dim3(tpb), 0, gs,
                             (const SweepParams*)ws->dev, ws->S, ws->cand);
          g = check_hip(hipGetLastError(), "slice screen launch");
        }
      }
      if (g == GW_OK) g = eval_rows(ctx, ws, k, a, gs);
      if (g == GW_OK && fused) {
        hipLaunchKernelGGL(k_sweep_step, dim3(blocks), dim3(tpb), 0, gs, (const SweepParams*)ws->dev, ws->S,
                           (const double*)ws->cand_logl, ws->cand, r & 1);
        g = check_hip(hipGetLastError(), "slice step launch");
      } else if (g == GW_OK) {
        hipLaunchKernelGGL(k_sweep_update, dim3(blocks), dim3(tpb), 0, gs, (const SweepParams*)ws->dev, ws->S,
                           (const double*)ws->cand_logl);
        g = check_hip(hipGetLastError(), "slice update launch");
      }
      if (g == GW_OK && a.cache)
        g = launch_wmom_build(ctx, ctx->coef, 2 * k, ws->S.build_list, ws->S.counts + 2, k, 2, ws->S.build_src,
                              a.prec, ws->wc, gs);
    }
    return g;
  };
  // the heterodyned rounds all evaluate the same 2k candidate rows: their
  // argument block is written once here instead of by every round
  struct Unpin {
    gw_ctx* c = nullptr;
    ~Unpin() {
      if (c) het_unpin_args(c);
    }
  } unpin;
  const bool pin = a.like == GW_HET && a.marg != GW_MARG_PHASE_TIME;
  if (s == GW_OK && pin) {
    s = het_pin_args(ctx, ws->cand, 2 * k, ws->cand_logl, st);
    if (s == GW_OK) unpin.c = ctx;
  }
  if (s == GW_OK && a.use_graph) s = slice_graph(ctx, ws, k, a, fused, pin, group);
  int cur = 0, prev = -1;
  for (int rounds = 0; s == GW_OK && rounds < max_rounds; rounds += 4) {
    if (a.use_graph) s = check_hip(hipGraphLaunch(ws->exec, st), "slice graph launch");
    else s = group(st);
    if (s != GW_OK) break;
    // a group's last round (r = 3) counts into n_active[1] when fused
    s = check_hip(hipMemcpyAsync(ws->h_active + cur, ws->S.n_active + (fused ? 1 : 0), sizeof(int32_t),
                                 hipMemcpyDeviceToHost, st),
                  "copy");
    if (s == GW_OK) s = check_hip(hipEventRecord(ws->ev[cur], st), "slice event");
    if (s != GW_OK) break;
    if (prev >= 0) {
      s = check_hip(hipEventSynchronize(ws->ev[prev]), "slice round sync");
      if (s == GW_OK && ws->h_active[prev] == 0) break;  // the group just queued only idles
    }
    prev = cur;
    cur ^= 1;
  }
  if (s != GW_OK) return s;
  hipLaunchKernelGGL(k_sweep_finish, dim3(blocks), dim3(tpb), 0, st, (const SweepParams*)ws->dev, ws->S, a.n_evals,
                     a.status);
  s = check_hip(hipGetLastError(), "slice finish launch");
  if (s == GW_OK && a.screen_stats) {
    s = check_hip(hipMemcpyAsync(ws->h_kinds + 3, ws->S.scr_tot, 3 * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, st), "copy");
    if (s == GW_OK) s = check_hip(hipStreamSynchronize(st), "slice sync");
    if (s == GW_OK)
      for (int i = 0; i < 3; ++i) a.screen_stats[i] = (int64_t)ws->h_kinds[3 + i];
  }
  if (s == GW_OK && a.eval_kinds) {
    if (!a.cache) {
      a.eval_kinds[0] = a.eval_kinds[1] = a.eval_kinds[2] = -1;  // not counted without the cache
      return GW_OK;
    }
    s = check_hip(hipMemcpyAsync(ws->h_kinds, ws->S.kind_tot, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                 st), "copy");
    if (s == GW_OK) s = check_hip(hipStreamSynchronize(st), "slice sync");
    if (s == GW_OK)
      for (int i = 0; i < 3; ++i) a.eval_kinds[i] = (int64_t)ws->h_kinds[i];
  }
  return s;
}

extern "C" {

gw_status slice_step(gw_ctx* ctx, const gw_slice_args* a, void* stream) {
  if (!ctx || !a) return set_error(GW_EINVAL, "slice_step: null argument");
  if (a->k == 0) return GW_OK;
  gw_status s = check_sweep("slice_step", a->k, a->x, a->logl, a->w, a->max_out, a->max_shrink, a->like, a->marg, ctx);
  if (s != GW_OK || a->k == 0) return s;
  if (!a->block || !a->chol) return set_error(GW_EINVAL, "slice_step: null pointer");
  SweepParams P{};
  int used = 0;
  s = set_block("slice_step", P, 0, a->block, a->block_dim, a->chol, a->block_dim, &used);
  if (s != GW_OK) return s;
  P.nb = 1;
  P.w = a->w;
  P.logl_star = a->logl_star;
  P.max_out = a->max_out;
  P.max_shrink = a->max_shrink;
  P.seed = a->seed;
  P.counter = a->counter;
  P.uniforms = a->uniforms;
  P.k = a->k;
  P.x = a->x;
  P.logl = a->logl;
  P.lists = a->like == GW_FULL && a->marg == GW_MARG_PHASE_DIST;
  s = cube_map(ctx, a->marg, &P.cm);
  if (s == GW_OK) s = set_screen("slice_step", ctx, a->mlp, a->margin, a->audit_frac, P);
  if (s == GW_OK) s = set_record("slice_step", a->rec_x, a->rec_logl, a->rec_cap, a->rec_count, P);
  if (s != GW_OK) return s;
  const int32_t graph = a->use_graph;
  const SweepCall c{a->like, a->marg, a->prec, graph, a->n_evals, a->status, 0, nullptr, P.lists,
                    P.screen ? a->mlp : nullptr, a->screen_stats};
  return run_sweep(ctx, P, c, (hipStream_t)stream);
}

gw_status slice_sweep(gw_ctx* ctx, const gw_sweep_args* a, void* stream) {
  if (!ctx || !a) return set_error(GW_EINVAL, "slice_sweep: null argument");
  if (a->k == 0) return GW_OK;
  gw_status s = check_sweep("slice_sweep", a->k, a->x, a->logl, a->w, a->max_out, a->max_shrink, a->like, a->marg,
                            ctx);
  if (s != GW_OK || a->k == 0) return s;
  if (a->n_blocks < 1 || a->n_blocks > kMaxBlocks) return set_error(GW_EINVAL, "slice_sweep: n_blocks 1..16");
  if (!a->block_dim || !a->block || !a->chol) return set_error(GW_EINVAL, "slice_sweep: null pointer");
  if (a->counter > UINT64_MAX - (uint64_t)a->n_blocks)
    return set_error(GW_EINVAL, "slice_sweep: counter + n_blocks overflows");
  SweepParams P{};
  int used = 0;
  for (int b = 0; b < a->n_blocks; ++b) {
    s = set_block("slice_sweep", P, b, a->block + b * GW_MAX_BLOCK, a->block_dim[b],
                  a->chol + b * GW_MAX_BLOCK * GW_MAX_BLOCK, GW_MAX_BLOCK, &used);
    if (s != GW_OK) return s;
  }
  P.nb = a->n_blocks;
  P.w = a->w;
  P.logl_star = a->logl_star;
  P.max_out = a->max_out;
  P.max_shrink = a->max_shrink;
  P.seed = a->seed;
  P.counter = a->counter;
  P.uniforms = nullptr;
  P.k = a->k;
  P.x = a->x;
  P.logl = a->logl;
  if (a->use_cache) {
    if (a->like != GW_FULL || a->marg != GW_MARG_PHASE_DIST)
      return set_error(GW_ENOTSUP, "slice_sweep: the waveform cache is for like=GW_FULL, marg=GW_MARG_PHASE_DIST");
    // kind of each block from its coordinates: psi and iota only change the
    // projection; sky position and t_c also change the delays; anything else
    // changes the waveform
    for (int b = 0; b < P.nb; ++b) {
      bool proj = true, extr = true;
      for (int i = 0; i < P.bd[b]; ++i) {
        const int j = P.block[b][i];
        proj = proj && (j == 6 || j == 9);
        extr = extr && j >= 6;
      }
      P.kind[b] = proj ? 2 : extr ? 1 : 0;
    }
    P.cache = 1;
    P.n_det = ctx->n_det;
  }
  P.lists = a->like == GW_FULL && a->marg == GW_MARG_PHASE_DIST;
  s = cube_map(ctx, a->marg, &P.cm);
  if (s == GW_OK) s = set_screen("slice_sweep", ctx, a->mlp, a->margin, a->audit_frac, P);
  if (s == GW_OK) s = set_record("slice_sweep", a->rec_x, a->rec_logl, a->rec_cap, a->rec_count, P);
  if (s != GW_OK) return s;
  const int32_t graph = a->use_graph;
  const SweepCall c{a->like, a->marg, a->prec, graph, a->n_evals, a->status, P.cache, a->eval_kinds, P.lists,
                    P.screen ? a->mlp : nullptr, a->screen_stats};
  return run_sweep(ctx, P, c, (hipStream_t)stream);
}

gw_status gw_set_sky_frame(gw_ctx* ctx, int32_t frame, int32_t det_a, int32_t det_b, int32_t det_time) {
  if (!ctx) return set_error(GW_EINVAL, "gw_set_sky_frame: ctx is NULL");
  if (frame != 0 && frame != 1) return set_error(GW_EINVAL, "gw_set_sky_frame: frame must be 0 or 1");
  if (frame == 0) {
    if (det_time) return set_error(GW_EINVAL, "gw_set_sky_frame: det_time needs the detector frame");
    ctx->sky_frame = 0;
    ctx->sky_det_time = 0;
    return GW_OK;
  }
  if (det_a < 0 || det_b < 0 || det_a >= ctx->n_det || det_b >= ctx->n_det || det_a == det_b)
    return set_error(GW_EINVAL, "gw_set_sky_frame: two distinct detectors 0 .. %d", ctx->n_det - 1);
  const double* ra = ctx->geom.pos[det_a];
  const double* rb = ctx->geom.pos[det_b];
  const double d2 = (rb[0] - ra[0]) * (rb[0] - ra[0]) + (rb[1] - ra[1]) * (rb[1] - ra[1]) +
                    (rb[2] - ra[2]) * (rb[2] - ra[2]);
  if (!(d2 > 1.0)) return set_error(GW_EINVAL, "gw_set_sky_frame: the two detectors are at the same place");
  if (det_time != 0 && det_time != 1) return set_error(GW_EINVAL, "gw_set_sky_frame: det_time must be 0 or 1");
  ctx->sky_frame = 1;
  ctx->sky_a = det_a;
  ctx->sky_b = det_b;
  ctx->sky_det_time = det_time;
  return GW_OK;
}

gw_status gw_prior_transform_marg(gw_ctx* ctx, const double* x, int64_t n, int32_t marg, double* theta,
                                  void* stream) {
  if (!ctx) return set_error(GW_EINVAL, "gw_prior_transform: ctx is NULL");
  if (n < 0) return set_error(GW_EINVAL, "gw_prior_transform: n < 0");
  if (marg != GW_MARG_PHASE_DIST && marg != GW_MARG_PHASE_TIME)
    return set_error(GW_EINVAL, "gw_prior_transform: marg must be GW_MARG_PHASE_DIST or GW_MARG_PHASE_TIME");
  if (n == 0) return GW_OK;
  if (!x || !theta) return set_error(GW_EINVAL, "gw_prior_transform: null pointer");
  CubeMap cm;
  gw_status s = cube_map(ctx, marg, &cm);
  if (s == GW_OK) s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  hipLaunchKernelGGL(k_prior_transform, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, x, n,
                     cm, theta);
  return check_hip(hipGetLastError(), "prior transform launch");
}

gw_status gw_prior_transform(gw_ctx* ctx, const double* x, int64_t n, double* theta, void* stream) {
  return gw_prior_transform_marg(ctx, x, n, GW_MARG_PHASE_DIST, theta, stream);
}

}  // extern "C"

static gw_status slice_ws(gw_ctx* ctx, int64_t k, gw_slice_ws** out) {
  gw_slice_ws*& ws = ctx->slice;
  if (!ws) {
    ws = new (std::nothrow) gw_slice_ws();
    if (!ws) return set_error(GW_ENOMEM, "slice workspace");
    if (hipHostMalloc((void**)&ws->h_active, 2 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
      return set_error(GW_ENOMEM, "slice pinned flag");
    for (int i = 0; i < 2; ++i)
      if (hipEventCreateWithFlags(&ws->ev[i], hipEventDisableTiming) != hipSuccess)
        return set_error(GW_EDEVICE, "slice events");
    if (hipHostMalloc((void**)&ws->h_kinds, 6 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
      return set_error(GW_ENOMEM, "slice pinned counters");
    if (hipMalloc((void**)&ws->dev, sizeof(SweepParams)) != hipSuccess) return set_error(GW_ENOMEM, "slice parameters");
  }
  if (ws->cap >= k) {
    *out = ws;
    return GW_OK;
  }
  if (ws->mem) (void)hipFree(ws->mem);
  ws->mem = nullptr;
  ws->cap = 0;
  // doubles: t_lo, t_hi, d[kMaxBlock], cand_t[2], cand[26], cand_logl[2], zrow[2][2 kMaxDet],
  // zc[3][2 kMaxDet], ucand[2][11], pred[2];
  // ints: flags, n_out[2], n_shrink, n_evals, slot_ok[2], cur, tot_evals, n_caps, rkind[2], zsrc[2],
  // build_list, build_src, dirty, slow_rows[2], stream_rows[2], scr[2], side_tests[2], then the two active
  // counters and the three list counts
  const size_t nd = (size_t)k * (1 + 1 + kMaxBlock + 2 + 26 + 2 + 4 * kMaxDet + 6 * kMaxDet + 2 * kSliceDim + 2);
  const size_t ni = (size_t)k * (1 + 2 + 1 + 1 + 2 + 3 + 2 + 2 + 1 + 1 + 1 + 2 + 2 + 2 + 2) + 5;
  char* m = nullptr;
  // six 64-bit counters first (evaluation kinds, prescreen counts), then the doubles and the ints
  gw_status s = check_hip(hipMalloc((void**)&m, 64 + nd * sizeof(double) + ni * sizeof(int32_t)), "slice workspace");
  if (s != GW_OK) return s;
  ws->S.kind_tot = (unsigned long long*)m;
  ws->S.scr_tot = ws->S.kind_tot + 3;
  double* dp = (double*)(m + 64);
  ws->S.t_lo = dp; dp += k;
  ws->S.t_hi = dp; dp += k;
  ws->S.d = dp; dp += k * kMaxBlock;
  ws->S.cand_t = dp; dp += 2 * k;
  ws->cand = dp; dp += 26 * k;
  ws->cand_logl = dp; dp += 2 * k;
  ws->S.zrow = dp; dp += 4 * kMaxDet * k;
  ws->S.zc = dp; dp += 6 * kMaxDet * k;
  ws->S.ucand = dp; dp += 2 * kSliceDim * k;
  ws->S.pred = dp; dp += 2 * k;
  int32_t* ip = (int32_t*)dp;
  ws->S.flags = ip; ip += k;
  ws->S.n_out = ip; ip += 2 * k;
  ws->S.n_shrink = ip; ip += k;
  ws->S.n_evals = ip; ip += k;
  ws->S.slot_ok = ip; ip += 2 * k;
  ws->S.cur = ip; ip += k;
  ws->S.tot_evals = ip; ip += k;
  ws->S.n_caps = ip; ip += k;
  ws->S.rkind = ip; ip += 2 * k;
  ws->S.zsrc = ip; ip += 2 * k;
  ws->S.build_list = ip; ip += k;
  ws->S.build_src = ip; ip += k;
  ws->S.dirty = ip; ip += k;
  ws->S.slow_rows = ip; ip += 2 * k;
  ws->S.stream_rows = ip; ip += 2 * k;
  ws->S.scr = ip; ip += 2 * k;
  ws->S.side_tests = ip; ip += 2 * k;
  ws->S.n_active = ip; ip += 2;
  ws->S.counts = ip;
  ws->mem = m;
  ws->cap = k;
  *out = ws;
  return GW_OK;
}

// Waveform cache of k slots (grown on demand; at most 64 GiB).
static gw_status slice_wcache(gw_ctx* ctx, gw_slice_ws* ws, int64_t k) {
  const int64_t f2 = wmom_slot_f2(ctx);
  if (ws->wc && ws->cap_wc >= k && ws->slot_f2 == f2) return GW_OK;
  if ((double)k * (double)f2 * sizeof(float2) > 64.0 * (1ull << 30))
    return set_error(GW_EINVAL, "slice_sweep: waveform cache of %lld chains x %lld bins exceeds 64 GiB",
                     (long long)k, (long long)f2);
  if (ws->wc) (void)hipFree(ws->wc);
  ws->wc = nullptr;
  ws->cap_wc = 0;
  gw_status s = check_hip(hipMalloc((void**)&ws->wc, (size_t)k * f2 * sizeof(float2)), "waveform cache");
  if (s != GW_OK) return s;
  ws->cap_wc = k;
  ws->slot_f2 = f2;
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
  if (ws->wc) (void)hipFree(ws->wc);
  if (ws->dev) (void)hipFree(ws->dev);
  if (ws->h_active) (void)hipHostFree(ws->h_active);
  if (ws->h_kinds) (void)hipHostFree(ws->h_kinds);
  for (hipEvent_t e : ws->ev)
    if (e) (void)hipEventDestroy(e);
  delete ws;
  ctx->slice = nullptr;
}
}  // namespace gw
