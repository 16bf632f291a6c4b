// Heterodyned (relative-binning) likelihood, Sec. III.D.
//
// Set-up (once per reference parameters theta0): bin edges of equal maximum
// phase change on the host, then on the device the reference phase at the
// edges and the per-detector summary data A0, A1 (data x reference) and
// B0, B1 (reference norm) per bin, by segmented sums over the fine grid with a
// fixed-order workgroup reduction.
//
// Evaluation: one lane per proposal, edge records wave-uniform (scalar loads).
// For TaylorF2 without a cut-off the ratio r_i = h_i / h0_i at an edge is
// (A P_i / A0 P0_i) exp(-2 pi i (Phi_i - Phi0_i)); the complex prefactor is
// pulled out of the bin sums, so per edge a lane evaluates the FP64 phase
// difference per detector, one phasor each, and the linear-in-bin contraction
// with the summary data.  Work arrives as a device-resident list of
// (row offset, count) sub-batches; a persistent grid of waves walks 64-row
// tiles of that list, so one launch (and one captured hipGraph) serves any
// sub-batch layout.  The distance marginal is evaluated inside the same wave.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <vector>

#include "gw_ctx.h"
#include "gw_hetplan.h"
#include "gw_tgrid.h"

// Device-resident arguments of the work-list kernels; a one-thread kernel
// writes them before each launch so that a captured graph can be replayed
// with new buffers.
struct HetArgs {
  const double* theta;
  const int64_t* subs;  // (row offset, count) pairs
  double* logl;
  double* coef;         // per-row coefficients [C_NCOEF][ld]
  double* zbuf;         // per-row (|Z_1|, <h|h>_1) [2][ld] for the distance marginal
  double* part;         // per-row partial sums [edge chunk][3 n_det][ld]
  int64_t n_rows;
  int64_t ld;
  int32_t n_sub;
  int32_t pad;
  double* zcplx;        // or NULL: per-row (Re Z, Im Z, <h|h>) [3][ld] for post-hoc reconstruction
};

struct gw_het_state {
  int n_bins = 0;
  int n_edges = 0;
  int rs = 0;                    // record stride (doubles)
  double* rec = nullptr;         // [n_edges][rs]
  std::vector<double> f_edges;   // host copy
  std::vector<double> theta0;
  double ap0_inv_re[gw::kMaxDet] = {0};
  double ap0_inv_im[gw::kMaxDet] = {0};
  double hh0[gw::kMaxDet] = {0};  // sum_b B0_b / 2 per detector (unit-phasor <h|h> constant)
  // work-list machinery
  HetArgs* args = nullptr;       // device
  int64_t* tile_pre = nullptr;   // device [max_sub + 1]
  int64_t* subs_single = nullptr;  // device [2]
  int max_sub = 0;
  // launch shape of the evaluation kernel
  int wpb = 4;                   // waves per workgroup
  int grid = 0;                  // workgroups (0 = heuristic)
  int ech = 0;                   // edge chunks (0 = heuristic)
  int64_t n_rows_last = 0;       // rows of the batch being enqueued (selects the distance form)
  // a caller that evaluates the same single batch (theta, rows, logl) many
  // times in a row writes the argument block once (het_pin_args); meanwhile
  // matching calls launch no k_set_args
  bool args_pinned = false;
  const double* pin_theta = nullptr;
  const double* pin_logl = nullptr;
  int64_t pin_rows = 0;
  // time marginal: row-independent tables for the current grid (built on
  // first use): per block b < n_blk the edges [bs[b], bs[b + 1]) in it, per
  // edge the Chebyshev values T_m(s_e) of its offset in the block (m < tm_K)
  // and the powers sigma_e^m of its bin width about the widths' centre
  // (m < tm_mh), and the moment kernel's chunks (gw_hetplan.h)
  double* tm_tab = nullptr;      // [n_edges][tm_K + tm_mh]
  // bs [n_blk + 1], then the plan: e0 [nch + 1], blo, bhi, sfirst, slast
  // [nch] each, then per cut block fb, fs, fc [tm_nsplit] each
  int32_t* tm_idx = nullptr;
  int tm_blk = 0, tm_nblk = 0, tm_mh = 0, tm_nch = 0, tm_nch_req = -1, tm_K = 0;
  int tm_nslot = 0, tm_nsplit = 0;  // piece slots and cut blocks of the plan
  double tm_hw = 0.0;            // half-range of the bin widths (fine bins)
  double tm_umax = -1.0;         // the window's largest |u| the norm series was sized for
  int64_t tm_c2 = 0;             // smallest + largest bin width (fine bins)
};

struct GraphKey {
  int marg, prec, wpb, grid, n_ech, sliced;
  bool operator<(const GraphKey& o) const {
    return std::tie(marg, prec, wpb, grid, n_ech, sliced) < std::tie(o.marg, o.prec, o.wpb, o.grid, o.n_ech, o.sliced);
  }
};

struct gw_graph_cache {
  std::map<GraphKey, hipGraphExec_t> exec;
  std::map<GraphKey, hipGraph_t> graph;
  hipStream_t cap_stream = nullptr;
  double last_instantiate_ms = 0.0;
};

namespace gw {

constexpr int kMaxSub = 1 << 16;

// Record layout of one edge e (bin e-1 data rides along with edge e).
__host__ __device__ constexpr int het_rs(int nd) { return 6 + 7 * nd; }
enum HetRec { H_X = 0, H_X2 = 1, H_XM5 = 2, H_LNF = 3, H_F = 4, H_PHI0 = 5 };  // then f dtau0_i (i >= 1)
__host__ __device__ constexpr int het_bin_off(int nd) { return 5 + nd; }      // inv width, then 6 per det
// The 6 per-detector slots of edge e first receive the summary data of bin e
// (between edges e-1 and e): A0 (re, im), A1 (re, im), B0, 2 B1.  The set-up
// then rewrites them as per-edge weights of the summed-by-parts bin sums
// (see k_het): C_e = R_e + L_{e+1} (re, im), R_e (re, im), B0_e / 2, 0, with
// R_e = A0_e / 2 + A1_e / w_e and L_e = A0_e / 2 - A1_e / w_e (w_e the width
// of bin e; R_0 = L_{n+1} = 0, B0_0 = 0).

// ---------------------------------------------------------------------------
// Set-up kernels

__global__ void k_het_edges(const double* __restrict__ bins, int bin_rs, const int64_t* __restrict__ edge_idx,
                            int n_edges, int nd, const double* __restrict__ coef0, TrigConsts T, int64_t k0,
                            double df, double* __restrict__ rec) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edges) return;
  const int rs = het_rs(nd);
  const int64_t k = edge_idx[e];
  const double* b = bins + k * bin_rs;
  PhaseCoef c;
  c.a0 = coef0[C_A0]; c.a2 = coef0[C_A2]; c.a3 = coef0[C_A3]; c.a4 = coef0[C_A4];
  c.a5 = coef0[C_A5]; c.a6 = coef0[C_A6]; c.a7 = coef0[C_A7]; c.a8 = coef0[C_A8];
  c.a10 = coef0[C_A10]; c.a12 = coef0[C_A12]; c.b5 = coef0[C_B5]; c.b6 = coef0[C_B6];
  const double f = (double)(k0 + k) * df;
  double* r = rec + (int64_t)e * rs;
  r[H_X] = b[0];
  r[H_X2] = b[1];
  r[H_XM5] = b[2];
  r[H_LNF] = b[3];
  r[H_F] = f;
  r[H_PHI0] = phase_cycles(c, b[0], b[1], b[2], b[3]);
  for (int i = 1; i < nd; ++i) r[H_PHI0 + i] = f * coef0[C_DT1 + i - 1];
  const int bo = het_bin_off(nd);
  if (e > 0) {
    const double fl = (double)(k0 + edge_idx[e - 1]) * df;
    r[bo] = 1.0 / (f - fl);
  } else {
    for (int j = bo; j < rs; ++j) r[j] = 0.0;
  }
  (void)T;
}

// One workgroup per (bin, detector): segmented sums over the fine bins of the
// bin with a fixed-order LDS tree.
__global__ void __launch_bounds__(256) k_het_summary(const double* __restrict__ bins, int bin_rs,
                                                     const double* __restrict__ hw, int64_t n_freq,
                                                     const int64_t* __restrict__ edge_idx, int n_bins,
                                                     const double* __restrict__ coef0, TrigConsts T, int64_t k0,
                                                     double df, double* __restrict__ rec, int nd) {
  const int b = blockIdx.x;
  const int i = blockIdx.y;
  const int64_t lo = edge_idx[b];
  const int64_t hi = edge_idx[b + 1];
  const int64_t stop = (b == n_bins - 1) ? hi + 1 : hi;
  const double fc = 0.5 * ((double)(k0 + lo) + (double)(k0 + hi)) * df;
  PhaseCoef c;
  c.a0 = coef0[C_A0]; c.a2 = coef0[C_A2]; c.a3 = coef0[C_A3]; c.a4 = coef0[C_A4];
  c.a5 = coef0[C_A5]; c.a6 = coef0[C_A6]; c.a7 = coef0[C_A7]; c.a8 = coef0[C_A8];
  c.a10 = coef0[C_A10]; c.a12 = coef0[C_A12]; c.b5 = coef0[C_B5]; c.b6 = coef0[C_B6];
  const double dt = i == 0 ? 0.0 : coef0[C_DT1 + i - 1];
  const double apr = coef0[C_APRE + i], api = coef0[C_APIM + i];
  const double ap2 = apr * apr + api * api;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t k = lo + threadIdx.x; k < stop; k += blockDim.x) {
    const double* r = bins + k * bin_rs;
    const double f = (double)(k0 + k) * df;
    const double ph = phase_cycles(c, r[0], r[1], r[2], r[3]) + f * dt;
    double s, co;
    sincos_cycles(ph, T, &s, &co);
    // 4 df d* h0 / S = u_ik (A P0_i) exp(-2 pi i phi)
    const double ur = r[4 + 2 * i], ui = r[5 + 2 * i];
    const double gr = apr * co + api * s, gi = api * co - apr * s;
    const double tr = ur * gr - ui * gi, ti = ur * gi + ui * gr;
    const double w = ap2 * hw[(int64_t)i * n_freq + k];
    const double dfc = f - fc;
    acc[0] += tr;
    acc[1] += ti;
    acc[2] += tr * dfc;
    acc[3] += ti * dfc;
    acc[4] += w;
    acc[5] += w * dfc;
  }
  __shared__ double red[6][256];
  for (int j = 0; j < 6; ++j) red[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int j = 0; j < 6; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* r = rec + (int64_t)(b + 1) * het_rs(nd) + het_bin_off(nd) + 1 + 6 * i;
    r[0] = red[0][0];
    r[1] = red[1][0];
    r[2] = red[2][0];
    r[3] = red[3][0];
    r[4] = red[4][0];
    r[5] = 2.0 * red[5][0];  // 2 B1
  }
}

// ---------------------------------------------------------------------------
// Work-list kernels

// Writes the argument block and the prefix sums of 64-row tiles per
// sub-batch (pre[s] = tiles before sub-batch s, pre[n_sub] = all tiles) in one
// launch of 256 threads.  ``subs`` is read from the device; a single batch
// (subs_single != NULL) is described by (0, single_n) without reading it back.
__global__ void __launch_bounds__(256) k_set_args(HetArgs* a, const double* theta, const int64_t* subs, double* logl,
                                                  double* coef, double* zbuf, double* part, int64_t n_rows,
                                                  int32_t n_sub, int64_t* subs_single, int64_t single_n,
                                                  int64_t* __restrict__ pre, double* zcplx) {
  if (threadIdx.x == 0) {
    a->zcplx = zcplx;
    a->theta = theta;
    a->subs = subs;
    a->logl = logl;
    a->coef = coef;
    a->zbuf = zbuf;
    a->part = part;
    a->n_rows = n_rows;
    a->ld = n_rows;
    a->n_sub = n_sub;
    a->pad = 0;
    if (subs_single) {
      subs_single[0] = 0;
      subs_single[1] = single_n;
    }
  }
  if (subs_single) {
    if (threadIdx.x == 0) {
      pre[0] = 0;
      pre[1] = n_rows > 0 ? (n_rows + 63) / 64 : 0;
    }
    return;
  }
  __shared__ int64_t acc[256];
  const int per = (n_sub + 255) / 256;
  const int s0 = threadIdx.x * per;
  const int s1 = min(s0 + per, n_sub);
  int64_t sum = 0;
  for (int q = s0; q < s1; ++q) {
    int64_t cnt = subs[2 * q + 1];
    const int64_t off = subs[2 * q];
    if (off < 0 || off >= n_rows || cnt <= 0) cnt = 0;
    else if (cnt > n_rows - off) cnt = n_rows - off;
    sum += (cnt + 63) / 64;
  }
  acc[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int j = 0; j < 256; ++j) {
      const int64_t v = acc[j];
      acc[j] = run;
      run += v;
    }
    pre[n_sub] = run;
  }
  __syncthreads();
  int64_t run = acc[threadIdx.x];
  for (int q = s0; q < s1; ++q) {
    pre[q] = run;
    int64_t cnt = subs[2 * q + 1];
    const int64_t off = subs[2 * q];
    if (off < 0 || off >= n_rows || cnt <= 0) cnt = 0;
    else if (cnt > n_rows - off) cnt = n_rows - off;
    run += (cnt + 63) / 64;
  }
}

// Tile t of the work list -> (first row, one-past-last row); returns false
// for an empty tile.
__device__ inline bool tile_rows(const HetArgs* __restrict__ ab, const int64_t* __restrict__ pre, int64_t t,
                                 int64_t* row0, int64_t* row_end) {
  int lo = 0, hi = ab->n_sub;  // invariant pre[lo] <= t < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= t) lo = mid;
    else hi = mid;
  }
  const int64_t off = ab->subs[2 * lo];
  int64_t cnt = ab->subs[2 * lo + 1];
  if (cnt > ab->n_rows - off) cnt = ab->n_rows - off;
  *row0 = off + (t - pre[lo]) * 64;
  *row_end = off + cnt;
  return *row0 < *row_end;
}

// Per-row prologue over the work list (same tiles as the evaluation kernel).
__global__ void __launch_bounds__(256) k_het_prologue(const HetArgs* __restrict__ ab,
                                                      const int64_t* __restrict__ pre, int marg, Geom geom) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const int64_t wid = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * wpb;
  const int64_t total = pre[ab->n_sub];
  const int64_t ld = ab->ld;
  for (int64_t t = wid; t < total; t += nwaves) {
    int64_t row0, row_end;
    if (!tile_rows(ab, pre, t, &row0, &row_end)) continue;
    const int64_t row = row0 + lane;
    if (row < row_end) prologue(ab->theta + row * 13, marg, geom, ab->coef + row, ld);
  }
}

struct HetConst {
  double ap0_inv_re[kMaxDet];
  double ap0_inv_im[kMaxDet];
  double hh0[kMaxDet];
  double dd;
};

template <int PREC>
__device__ inline void het_phasor(double r, const TrigConsts& T, double* gr, double* gi) {
  if (PREC == 0) {
    double s, c;
    sincos_cycles(r, T, &s, &c);
    *gr = c;
    *gi = -s;
  } else {
    const float t = (float)(r - rint(r));
    const double c = (double)__builtin_amdgcn_cosf(t);
    const double s = (double)__builtin_amdgcn_sinf(t);
    // One Newton step towards unit modulus: the hardware pair has |g|^2 about
    // 6e-8 below 1 on average, and the binned norm sums are quadratic in g.
    const double k = fma(-0.5, fma(c, c, s * s), 1.5);
    *gr = c * k;
    *gi = -s * k;
  }
}

// Binned sums of one (tile, edge chunk) work item.  The waves of a workgroup
// take consecutive tiles of the same edge chunk; the chunk's edge records are
// staged through LDS in pieces of up to kLdsEdges edges (coalesced copy by the
// whole workgroup, then wave-uniform broadcast reads).  Per lane the partial
// (Z_i, <h_i|h_i>) of the chunk's bins go to ab->part, without the
// (A P_i) / (A0 P0_i) prefactor.
constexpr int kLdsEdges = 128;

template <int ND, int PREC>
__global__ void __launch_bounds__(256) k_het(const HetArgs* __restrict__ ab, const int64_t* __restrict__ pre,
                                             const double* __restrict__ rec, int n_bins, int n_ech, TrigConsts T) {
  constexpr int RS = het_rs(ND);
  constexpr int BO = het_bin_off(ND);
  __shared__ double srec[kLdsEdges * RS];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int64_t total = pre[ab->n_sub];
  const int64_t groups = (total + wpb - 1) / wpb;
  const int64_t ld = ab->ld;
  const double* __restrict__ coef = ab->coef;
  const int per = (n_bins + n_ech - 1) / n_ech;

  for (int64_t q = blockIdx.x; q < groups * n_ech; q += gridDim.x) {
    const int ech = (int)(q % n_ech);
    const int64_t t = (q / n_ech) * wpb + wave;
    int64_t row0 = 0, row_end = 0;
    const bool has = t < total && tile_rows(ab, pre, t, &row0, &row_end);
    const int64_t row = row0 + lane;
    const bool active = has && row < row_end;
    const int64_t rr = active ? row : (has ? row0 : 0);
    const double* cf = coef + rr;
    PhaseCoef c;
    double dt[ND];
    dt[0] = 0.0;
    if (has) {
      c.a0 = cf[C_A0 * ld]; c.a2 = cf[C_A2 * ld]; c.a3 = cf[C_A3 * ld]; c.a4 = cf[C_A4 * ld];
      c.a5 = cf[C_A5 * ld]; c.a6 = cf[C_A6 * ld]; c.a7 = cf[C_A7 * ld]; c.a8 = cf[C_A8 * ld];
      c.a10 = cf[C_A10 * ld]; c.a12 = cf[C_A12 * ld]; c.b5 = cf[C_B5 * ld]; c.b6 = cf[C_B6 * ld];
#pragma unroll
      for (int i = 1; i < ND; ++i) dt[i] = cf[(C_DT1 + i - 1) * ld];
    }

    // bins (b0, b1] of this chunk (bin e lies between edges e - 1 and e) use edges b0 .. b1
    const int b0 = ech * per < n_bins ? ech * per : n_bins;
    const int b1 = b0 + per < n_bins ? b0 + per : n_bins;
    double zr[ND], zi[ND], hh[ND], pr[ND], pi[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      zr[i] = zi[i] = hh[i] = 0.0;
      pr[i] = pi[i] = 0.0;
    }
    const int e_last = b1 > b0 ? b1 : b0 - 1;  // empty chunk: no edges
    for (int e0 = b0; e0 <= e_last; e0 += kLdsEdges) {
      const int ne = e_last - e0 + 1 < kLdsEdges ? e_last - e0 + 1 : kLdsEdges;
      __syncthreads();
      for (int j = threadIdx.x; j < ne * RS; j += blockDim.x) srec[j] = rec[(int64_t)e0 * RS + j];
      __syncthreads();
      if (!has) continue;
      for (int el = 0; el < ne; ++el) {
        const int e = e0 + el;
        const double* r = srec + el * RS;
        const double d0 = phase_cycles(c, r[H_X], r[H_X2], r[H_XM5], r[H_LNF]) - r[H_PHI0];
        const double f = r[H_F];
        // weight of this edge in the chunk's bins (b0, b1]: C inside, the
        // left-edge part C - R at b0, the right-edge part R at b1 (uniform)
        const int side = e == b0 ? 1 : (e == b1 ? 2 : 0);
#pragma unroll
        for (int i = 0; i < ND; ++i) {
          const double di = i == 0 ? d0 : fma(f, dt[i], d0) - r[H_PHI0 + i];
          double gr, gi;
          het_phasor<PREC>(di, T, &gr, &gi);
          const double* w = r + BO + 1 + 6 * i;
          const double kr = side == 0 ? w[0] : (side == 1 ? w[0] - w[2] : w[2]);
          const double ki = side == 0 ? w[1] : (side == 1 ? w[1] - w[3] : w[3]);
          zr[i] = fma(kr, gr, fma(-ki, gi, zr[i]));
          zi[i] = fma(kr, gi, fma(ki, gr, zi[i]));
          // |r0|^2 = (1 + Re(g_e conj g_{e-1})) / 2 for unit phasors; the
          // constant half is added once per row by the combine kernel
          if (e > b0) hh[i] = fma(w[4], fma(gr, pr[i], gi * pi[i]), hh[i]);
          pr[i] = gr;
          pi[i] = gi;
        }
      }
    }
    if (active) {
      double* out = ab->part + (int64_t)ech * 3 * ND * ld + row;
#pragma unroll
      for (int i = 0; i < ND; ++i) {
        out[(3 * i) * ld] = zr[i];
        out[(3 * i + 1) * ld] = zi[i];
        out[(3 * i + 2) * ld] = hh[i];
      }
    }
  }
}

// Combine the edge-chunk partials of each row in chunk order, restore the
// prefactor (A P_i) / (A0 P0_i), sum the detectors and apply the plain or
// phase-marginalised epilogue (or stage |Z_1| and <h|h>_1 for the distance
// marginal).
// Finish one row from its per-detector sums (z_i, unit-phasor <h|h> part):
// restore the prefactor (A P_i) / (A0 P0_i), sum the detectors and apply the
// plain or phase-marginalised epilogue (or stage |Z_1| and <h|h>_1 for the
// distance marginal).
struct HetRow {
  double Zr, Zi, plain, hht;
  bool valid;
};

// A row's binned overlap, its plain real part and <h|h> from the summed edge
// partials (the heterodyne's per-detector ratio to the reference applied).
__device__ inline HetRow het_row(const HetArgs* __restrict__ ab, int64_t row, int nd, const double* zr,
                                 const double* zi, const double* hh, const HetConst& hc) {
  const int64_t ld = ab->ld;
  const double* cf = ab->coef + row;
  double Zr = 0.0, Zi = 0.0, plain = 0.0, hht = 0.0;
  for (int i = 0; i < nd; ++i) {
    const double ar = cf[(C_APRE + i) * ld], ai = cf[(C_APIM + i) * ld];
    const double qr = ar * hc.ap0_inv_re[i] - ai * hc.ap0_inv_im[i];
    const double qi = ar * hc.ap0_inv_im[i] + ai * hc.ap0_inv_re[i];
    const double wr = qr * zr[i] - qi * zi[i];
    const double wi = qr * zi[i] + qi * zr[i];
    plain += wr;
    Zr += wr;
    Zi += wi;
    hht += (qr * qr + qi * qi) * (hc.hh0[i] + hh[i]);
  }
  return HetRow{Zr, Zi, plain, hht, cf[C_VALID * ld] != 0.0};
}

__device__ inline void het_finish_row(const HetArgs* __restrict__ ab, int64_t row, int nd, int marg,
                                      const double* zr, const double* zi, const double* hh, const HetConst& hc) {
  const int64_t ld = ab->ld;
  const HetRow R = het_row(ab, row, nd, zr, zi, hh, hc);
  const double Zr = R.Zr, Zi = R.Zi, plain = R.plain, hht = R.hht;
  const bool valid = R.valid;
  const double zabs = sqrt(Zr * Zr + Zi * Zi);
  if (ab->zcplx) {
    ab->zcplx[row] = valid ? Zr : NAN;
    ab->zcplx[ld + row] = Zi;
    ab->zcplx[2 * ld + row] = hht;
  }
  if (marg == 2) {
    ab->zbuf[row] = valid ? zabs : -1.0;
    ab->zbuf[ld + row] = hht;
  } else {
    double out;
    if (!valid) out = -INFINITY;
    else if (marg == 0) out = -0.5 * hc.dd + plain - 0.5 * hht;
    else out = -0.5 * hc.dd - 0.5 * hht + log_i0(zabs);
    ab->logl[row] = out;
  }
}

// Large batches: one lane per row (coalesced over rows), the edge-chunk
// partials summed in chunk order.
__global__ void __launch_bounds__(256) k_het_combine(const HetArgs* __restrict__ ab, const int64_t* __restrict__ pre,
                                                     int nd, int n_ech, int marg, HetConst hc) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const int64_t wid = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * wpb;
  const int64_t total = pre[ab->n_sub];
  const int64_t ld = ab->ld;
  for (int64_t t = wid; t < total; t += nwaves) {
    int64_t row0, row_end;
    if (!tile_rows(ab, pre, t, &row0, &row_end)) continue;
    const int64_t row = row0 + lane;
    if (row >= row_end) continue;
    double zr[kMaxDet], zi[kMaxDet], hh[kMaxDet];
    for (int i = 0; i < nd; ++i) {
      zr[i] = zi[i] = hh[i] = 0.0;
      for (int e = 0; e < n_ech; ++e) {
        const double* p = ab->part + ((int64_t)e * 3 * nd + 3 * i) * ld + row;
        zr[i] += p[0];
        zi[i] += p[ld];
        hh[i] += p[2 * ld];
      }
    }
    het_finish_row(ab, row, nd, marg, zr, zi, hh, hc);
  }
}

// Small batches (and at most 64 edge chunks): one wave per row, lane e
// holding chunk e's partials, summed by a fixed shuffle tree, so that the
// loads of a row are issued together instead of one chain per thread.
__global__ void __launch_bounds__(256) k_het_combine_w(const HetArgs* __restrict__ ab,
                                                       const int64_t* __restrict__ pre, int nd, int n_ech, int marg,
                                                       HetConst hc) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const int64_t wid = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * wpb;
  const int64_t total = pre[ab->n_sub] * 64;
  const int64_t ld = ab->ld;
  for (int64_t it = wid; it < total; it += nwaves) {
    int64_t row0, row_end;
    if (!tile_rows(ab, pre, it >> 6, &row0, &row_end)) continue;
    const int64_t row = row0 + (it & 63);
    if (row >= row_end) continue;
    double zr[kMaxDet], zi[kMaxDet], hh[kMaxDet];
    for (int i = 0; i < nd; ++i) {
      double a = 0.0, b = 0.0, c = 0.0;
      if (lane < n_ech) {
        const double* p = ab->part + ((int64_t)lane * 3 * nd + 3 * i) * ld + row;
        a = p[0];
        b = p[ld];
        c = p[2 * ld];
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
      }
      zr[i] = a;
      zi[i] = b;
      hh[i] = c;
    }
    if (lane == 0) het_finish_row(ab, row, nd, marg, zr, zi, hh, hc);
  }
}

// Distance marginal over the work list, small batches: one wave per row
// (wave_dist_lse), which keeps many waves busy when there are few rows.
template <int PREC>
__global__ void __launch_bounds__(256) k_het_dist_w(const HetArgs* __restrict__ ab, const int64_t* __restrict__ pre,
                                                    const double* __restrict__ dtab, int n_dist, double dd,
                                                    const LogI0Consts* __restrict__ Cp) {
  const LogI0Consts& C = *Cp;
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const int64_t wid = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * wpb;
  const int64_t total = pre[ab->n_sub] * 64;
  const int64_t ld = ab->ld;
  for (int64_t it = wid; it < total; it += nwaves) {
    int64_t row0, row_end;
    if (!tile_rows(ab, pre, it >> 6, &row0, &row_end)) continue;
    const int64_t row = row0 + (it & 63);
    if (row >= row_end) continue;
    const double z1 = ab->zbuf[row];
    const double h1 = ab->zbuf[ld + row];
    if (z1 < 0.0) {
      if (lane == 0) ab->logl[row] = -INFINITY;
      continue;
    }
    const double v = PREC == 0 ? wave_dist_lse(z1, h1, dtab, n_dist, lane, C)
                               : wave_dist_lse_f32(z1, h1, dtab, n_dist, lane);
    if (lane == 0) ab->logl[row] = -0.5 * dd + v;
  }
}

// Small batches with the distance marginal: k_het_combine_w and k_het_dist_w
// in one launch (one wave per row), the row's |Z| and <h|h> passed on in
// registers; the same arithmetic, so the same log L.
template <int PREC>
__global__ void __launch_bounds__(256) k_het_combine_dist_w(const HetArgs* __restrict__ ab,
                                                            const int64_t* __restrict__ pre, int nd, int n_ech,
                                                            HetConst hc, const double* __restrict__ dtab, int n_dist,
                                                            const LogI0Consts* __restrict__ Cp) {
  const LogI0Consts& C = *Cp;
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const int64_t wid = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * wpb;
  const int64_t total = pre[ab->n_sub] * 64;
  const int64_t ld = ab->ld;
  for (int64_t it = wid; it < total; it += nwaves) {
    int64_t row0, row_end;
    if (!tile_rows(ab, pre, it >> 6, &row0, &row_end)) continue;
    const int64_t row = row0 + (it & 63);
    if (row >= row_end) continue;
    double zr[kMaxDet], zi[kMaxDet], hh[kMaxDet];
    for (int i = 0; i < nd; ++i) {
      double a = 0.0, b = 0.0, c = 0.0;
      if (lane < n_ech) {
        const double* p = ab->part + ((int64_t)lane * 3 * nd + 3 * i) * ld + row;
        a = p[0];
        b = p[ld];
        c = p[2 * ld];
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
      }
      zr[i] = a;
      zi[i] = b;
      hh[i] = c;
    }
    const HetRow R = het_row(ab, row, nd, zr, zi, hh, hc);
    const double z1 = R.valid ? sqrt(R.Zr * R.Zr + R.Zi * R.Zi) : -1.0, h1 = R.hht;
    if (lane == 0) {
      if (ab->zcplx) {
        ab->zcplx[row] = R.valid ? R.Zr : NAN;
        ab->zcplx[ld + row] = R.Zi;
        ab->zcplx[2 * ld + row] = R.hht;
      }
      ab->zbuf[row] = z1;
      ab->zbuf[ld + row] = h1;
    }
    if (z1 < 0.0) {
      if (lane == 0) ab->logl[row] = -INFINITY;
      continue;
    }
    const double v = PREC == 0 ? wave_dist_lse(z1, h1, dtab, n_dist, lane, C)
                               : wave_dist_lse_f32(z1, h1, dtab, n_dist, lane);
    if (lane == 0) ab->logl[row] = -0.5 * hc.dd + v;
  }
}

// Distance marginal over the work list, large batches: a workgroup per 64-row
// tile, lane = row, waves splitting the grid (block_dist_lse), so that grid
// records are scalar loads shared by 64 rows.
constexpr int64_t kDistRowsPerLane = 8192;  // batches from this size use the sliced form
constexpr int kHetDistWaves = 8;  // waves per 64-row tile in the sliced form

template <int PREC>
__global__ void __launch_bounds__(64 * kHetDistWaves) k_het_dist(const HetArgs* __restrict__ ab,
                                                                 const int64_t* __restrict__ pre,
                                                                 const double* __restrict__ dtab, int n_dist,
                                                                 double dd, const LogI0Consts* __restrict__ Cp) {
  const LogI0Consts& C = *Cp;
  __shared__ double red[kHetDistWaves * 64];
  const int lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  const int64_t tiles = pre[ab->n_sub];
  const int64_t ld = ab->ld;
  // one 64-row tile per workgroup iteration (uniform across the block)
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    int64_t row0 = 0, row_end = 0;
    const bool has = tile_rows(ab, pre, t, &row0, &row_end);
    const int64_t row = row0 + lane;
    const bool active = has && row < row_end;
    const int64_t rr = active ? row : (has ? row0 : 0);
    const double z1 = has ? ab->zbuf[rr] : 0.0;
    const double h1 = has ? ab->zbuf[ld + rr] : 0.0;
    const double v = block_dist_lse<PREC>(z1 < 0.0 ? 0.0 : z1, h1, dtab, n_dist, nw, red, C);
    if ((threadIdx.x >> 6) == 0 && active) ab->logl[row] = z1 < 0.0 ? -INFINITY : -0.5 * dd + v;
  }
}

// ---------------------------------------------------------------------------
// Host side

static void free_state(gw_het_state* h) {
  if (!h) return;
  if (h->tm_tab) (void)hipFree(h->tm_tab);
  if (h->tm_idx) (void)hipFree(h->tm_idx);
  if (h->rec) (void)hipFree(h->rec);
  if (h->args) (void)hipFree(h->args);
  if (h->tile_pre) (void)hipFree(h->tile_pre);
  if (h->subs_single) (void)hipFree(h->subs_single);
  delete h;
}

void het_free(gw_ctx* ctx) {
  free_state(ctx->het);
  ctx->het = nullptr;
}

static void graphs_clear(gw_graph_cache* g) {
  for (auto& kv : g->exec) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : g->graph) (void)hipGraphDestroy(kv.second);
  g->exec.clear();
  g->graph.clear();
}

void graphs_free(gw_ctx* ctx) {
  if (!ctx->graphs) return;
  graphs_clear(ctx->graphs);
  if (ctx->graphs->cap_stream) (void)hipStreamDestroy(ctx->graphs->cap_stream);
  delete ctx->graphs;
  ctx->graphs = nullptr;
}

// Edge indices of the bin grid (host, FP64); see heterodyne_setup in gwswig.h.
static std::vector<int64_t> make_edges(const Geom& g, int n_bins, int rule) {
  const int64_t n = g.n_freq;
  std::vector<double> f(n);
  for (int64_t k = 0; k < n; ++k) f[k] = (double)(g.k0 + k) * g.df;
  const double fmin = f[0], fmax = f[n - 1];
  std::vector<double> fe(n_bins + 1);
  if (rule == 0) {
    const double gam[5] = {-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0};
    std::vector<double> phi(n);
    for (int64_t k = 0; k < n; ++k) {
      double s = 0.0;
      for (double gg : gam) {
        const double fs = gg > 0 ? fmax : fmin;
        s += (gg > 0 ? 1.0 : -1.0) * pow(f[k] / fs, gg);
      }
      phi[k] = s;
    }
    int64_t k = 0;
    for (int j = 0; j <= n_bins; ++j) {
      const double y = phi[0] + j * (phi[n - 1] - phi[0]) / n_bins;
      while (k + 1 < n - 1 && phi[k + 1] <= y) ++k;
      if (y <= phi[0]) fe[j] = f[0];
      else if (y >= phi[n - 1]) fe[j] = f[n - 1];
      else fe[j] = f[k] + (y - phi[k]) * (f[k + 1] - f[k]) / (phi[k + 1] - phi[k]);
    }
  } else {
    for (int j = 0; j <= n_bins; ++j) fe[j] = fmin * pow(fmax / fmin, (double)j / n_bins);
  }
  std::vector<int64_t> idx(n_bins + 1);
  for (int j = 0; j <= n_bins; ++j) {
    int64_t v = (int64_t)rint((fe[j] - fmin) / (f[1 < n ? 1 : 0] - f[0] + (n > 1 ? 0.0 : 1.0)));
    idx[j] = std::min<int64_t>(std::max<int64_t>(v, 0), n - 1);
  }
  idx[0] = 0;
  idx[n_bins] = n - 1;
  std::sort(idx.begin(), idx.end());
  idx.erase(std::unique(idx.begin(), idx.end()), idx.end());
  return idx;
}

// Edge chunks per tile: enough (tile, chunk) items to give every SIMD a few
// waves at this batch size, at least 16 bins per chunk, at most 32 chunks.
// Default persistent grid of the evaluation kernel, in waves (measured best
// of 2048 .. 16384 at 65,536 rows and 500 bins).
constexpr int64_t kHetWaves = 16384;

static int het_ech(const gw_ctx* ctx, int64_t n_rows) {
  const int64_t nb = ctx->het->n_bins;
  if (ctx->het->ech > 0) return (int)std::min<int64_t>(ctx->het->ech, nb);
  // about one (tile, edge chunk) item per wave of the default grid, at most
  // 64 chunks (one lane each in the combine) of at least 8 edges: a
  // sampler's 250-row batch of 500 bins takes 31.2 us a call at 62 chunks
  // against 36.0 at 31
  const int64_t tiles = (n_rows + 63) / 64;
  int64_t e = (kHetWaves + tiles - 1) / tiles;
  const int64_t emax = std::max<int64_t>(1, std::min<int64_t>(64, nb / 8));
  e = std::max<int64_t>(1, std::min(e, emax));
  return (int)e;
}

template <int ND>
static gw_status launch_het_nd(gw_ctx* ctx, int marg, int prec, int n_ech, hipStream_t st) {
  gw_het_state* h = ctx->het;
  const TrigConsts T = make_trig_consts();
  const int tpb = 64 * h->wpb;
  int grid = h->grid;
  // 64 waves per CU (several rounds of the resident 20); small batches have
  // few items, and an idle grid still costs dispatch time
  if (grid <= 0) grid = (h->n_rows_last < kDistRowsPerLane ? 1024 : kHetWaves) / h->wpb;
  const int slot = prof_begin(ctx, st, 1);
  if (prec == GW_PREC_FP64)
    hipLaunchKernelGGL((k_het<ND, 0>), dim3(grid), dim3(tpb), 0, st, h->args, h->tile_pre, h->rec, h->n_bins, n_ech,
                       T);
  else
    hipLaunchKernelGGL((k_het<ND, 1>), dim3(grid), dim3(tpb), 0, st, h->args, h->tile_pre, h->rec, h->n_bins, n_ech,
                       T);
  prof_end(ctx, slot, st);
  (void)marg;
  return check_hip(hipGetLastError(), "heterodyne kernel launch");
}

// Queue the work-list sequence: tile scan, prologue, binned sums, combine
// (+ distance marginal).  Reads the device argument block only.
static gw_status enqueue_het(gw_ctx* ctx, int marg, int prec, int n_ech, hipStream_t st) {
  gw_het_state* h = ctx->het;
  const bool small = h->n_rows_last < kDistRowsPerLane;
  hipLaunchKernelGGL(k_het_prologue, dim3(small ? 32 : 256 * 4), dim3(256), 0, st, h->args, h->tile_pre, marg,
                     ctx->geom);
  gw_status s = check_hip(hipGetLastError(), "heterodyne prologue launch");
  if (s != GW_OK) return s;
  switch (ctx->n_det) {
    case 1: s = launch_het_nd<1>(ctx, marg, prec, n_ech, st); break;
    case 2: s = launch_het_nd<2>(ctx, marg, prec, n_ech, st); break;
    case 3: s = launch_het_nd<3>(ctx, marg, prec, n_ech, st); break;
    case 4: s = launch_het_nd<4>(ctx, marg, prec, n_ech, st); break;
    default: s = set_error(GW_ENOTSUP, "n_det not supported");
  }
  if (s != GW_OK) return s;
  HetConst hc;
  for (int i = 0; i < kMaxDet; ++i) {
    hc.ap0_inv_re[i] = h->ap0_inv_re[i];
    hc.ap0_inv_im[i] = h->ap0_inv_im[i];
    hc.hh0[i] = h->hh0[i];
  }
  hc.dd = ctx->dd;
  if (marg == 2 && h->n_rows_last < kDistRowsPerLane && n_ech <= 64) {
    if (prec == GW_PREC_MIXED)
      hipLaunchKernelGGL(k_het_combine_dist_w<1>, dim3(256 * 8), dim3(256), 0, st, h->args, h->tile_pre, ctx->n_det,
                         n_ech, hc, ctx->dist_tab, ctx->n_dist, ctx->i0c);
    else
      hipLaunchKernelGGL(k_het_combine_dist_w<0>, dim3(256 * 8), dim3(256), 0, st, h->args, h->tile_pre, ctx->n_det,
                         n_ech, hc, ctx->dist_tab, ctx->n_dist, ctx->i0c);
    return check_hip(hipGetLastError(), "heterodyne combine and distance marginal launch");
  }
  if (h->n_rows_last < kDistRowsPerLane && n_ech <= 64)
    hipLaunchKernelGGL(k_het_combine_w, dim3(256 * 8), dim3(256), 0, st, h->args, h->tile_pre, ctx->n_det, n_ech,
                       marg, hc);
  else
    hipLaunchKernelGGL(k_het_combine, dim3(256 * 4), dim3(256), 0, st, h->args, h->tile_pre, ctx->n_det, n_ech,
                       marg, hc);
  s = check_hip(hipGetLastError(), "heterodyne combine launch");
  if (s != GW_OK || marg != 2) return s;
  // large batches: lane = row (grid records are scalar loads shared by 64
  // rows); small batches: wave = row
  const bool sliced = h->n_rows_last >= kDistRowsPerLane;
  if (sliced && prec == GW_PREC_MIXED)
    hipLaunchKernelGGL(k_het_dist<1>, dim3(256 * 8), dim3(64 * kHetDistWaves), 0, st, h->args, h->tile_pre,
                       ctx->dist_tab, ctx->n_dist, ctx->dd, ctx->i0c);
  else if (sliced)
    hipLaunchKernelGGL(k_het_dist<0>, dim3(256 * 8), dim3(64 * kHetDistWaves), 0, st, h->args, h->tile_pre,
                       ctx->dist_tab, ctx->n_dist, ctx->dd, ctx->i0c);
  else if (prec == GW_PREC_MIXED)
    hipLaunchKernelGGL(k_het_dist_w<1>, dim3(256 * 8), dim3(256), 0, st, h->args, h->tile_pre, ctx->dist_tab,
                       ctx->n_dist, ctx->dd, ctx->i0c);
  else
    hipLaunchKernelGGL(k_het_dist_w<0>, dim3(256 * 8), dim3(256), 0, st, h->args, h->tile_pre, ctx->dist_tab,
                       ctx->n_dist, ctx->dd, ctx->i0c);
  return check_hip(hipGetLastError(), "heterodyne distance marginal launch");
}

// Workspace for n_rows rows and the argument block; returns the edge-chunk count.
static gw_status het_prepare(gw_ctx* ctx, const double* theta, const int64_t* subs, int32_t n_sub, int64_t n_rows,
                             double* logl, bool single, int* n_ech, hipStream_t st, double* zcplx = nullptr) {
  gw_het_state* h = ctx->het;
  h->n_rows_last = n_rows;
  *n_ech = het_ech(ctx, n_rows);
  gw_status s = ensure_buffer(&ctx->coef, &ctx->coef_cap, (int64_t)C_NCOEF * n_rows, "coefficient workspace");
  if (s == GW_OK) s = ensure_buffer(&ctx->zbuf, &ctx->zbuf_cap, 2 * n_rows, "marginal workspace");
  if (s == GW_OK)
    s = ensure_buffer(&ctx->partial, &ctx->partial_cap, (int64_t)(*n_ech) * 3 * ctx->n_det * n_rows, "partials");
  if (s != GW_OK) return s;
  if (h->args_pinned) {
    if (single && !zcplx && theta == h->pin_theta && logl == h->pin_logl && n_rows == h->pin_rows) return GW_OK;
    h->args_pinned = false;  // the block is rewritten below
  }
  hipLaunchKernelGGL(k_set_args, dim3(1), dim3(256), 0, st, h->args, theta,
                     single ? (const int64_t*)h->subs_single : subs, logl, ctx->coef, ctx->zbuf, ctx->partial, n_rows,
                     single ? 1 : n_sub, single ? h->subs_single : (int64_t*)nullptr, single ? n_rows : (int64_t)0,
                     h->tile_pre, zcplx);
  return check_hip(hipGetLastError(), "argument kernel launch");
}

gw_status het_pin_args(gw_ctx* ctx, const double* theta, int64_t n, double* logl, hipStream_t st) {
  gw_het_state* h = ctx->het;
  if (!h) return set_error(GW_ESTATE, "heterodyne_setup has not been called");
  h->args_pinned = false;
  int n_ech = 1;
  gw_status s = het_prepare(ctx, theta, nullptr, 1, n, logl, true, &n_ech, st);
  if (s != GW_OK) return s;
  h->pin_theta = theta;
  h->pin_logl = logl;
  h->pin_rows = n;
  h->args_pinned = true;
  return GW_OK;
}

void het_unpin_args(gw_ctx* ctx) {
  if (ctx->het) ctx->het->args_pinned = false;
}

gw_status het_reserve(gw_ctx* ctx, int64_t n) {
  if (!ctx->het) return set_error(GW_ESTATE, "heterodyne_setup has not been called");
  const int n_ech = het_ech(ctx, n);
  gw_status s = ensure_buffer(&ctx->coef, &ctx->coef_cap, (int64_t)C_NCOEF * n, "coefficient workspace");
  if (s == GW_OK) s = ensure_buffer(&ctx->zbuf, &ctx->zbuf_cap, 2 * n, "marginal workspace");
  if (s == GW_OK) s = ensure_buffer(&ctx->partial, &ctx->partial_cap, (int64_t)n_ech * 3 * ctx->n_det * n, "partials");
  return s;
}

void het_shape_key(const gw_ctx* ctx, int32_t* wpb, int32_t* grid, int32_t* ech) {
  *wpb = ctx->het ? ctx->het->wpb : 0;
  *grid = ctx->het ? ctx->het->grid : 0;
  *ech = ctx->het ? ctx->het->ech : 0;
}

void het_tm_key(const gw_ctx* ctx, const void** tab, const void** idx, int32_t* nch, int32_t* nslot, int32_t* nsplit) {
  const gw_het_state* h = ctx->het;
  *tab = h ? h->tm_tab : nullptr;
  *idx = h ? h->tm_idx : nullptr;
  *nch = h ? h->tm_nch : 0;
  *nslot = h ? h->tm_nslot : 0;
  *nsplit = h ? h->tm_nsplit : 0;
}

// ---------------------------------------------------------------------------
// Time marginal on the binned likelihood (the appendix's direct sum on the
// heterodyned bins).  A shift t multiplies every edge phasor by
// exp(-2 pi i f_e t), so with per-row edge weights
//   W_e = sum_i q_i K_ie g_ie          (K the summed-by-parts overlap weights),
//   V_e = sum_i |q_i|^2 (B0_e / 2) g_ie conj(g_i,e-1)   (bin e's norm term),
// q_i = (A P_i) / (A0 P0_i), the binned overlap and norm at t_j are
//   Z(t_j)  = sum_e W_e exp(-2 pi i f_e t_j),
//   hh(t_j) = sum_i |q_i|^2 hh0_i + Re sum_e V_e exp(-2 pi i (f_e - f_e-1) t_j).
// The edges lie on the fine grid, so Z goes through the block moments of the
// full band's time marginal with W_e in place of the per-bin weights
// (gw_tgrid.hip); the widths f_e - f_e-1 = dk_e df span a short range, and
// exp(-2 pi i dk_e u) about the widths' centre c, dk_e = c + hw sigma_e, is a
// series in (2 pi hw u) sigma_e whose moments S_m = sum_e sigma_e^m V_e the
// grid kernel sums (tm_mh terms, the first dropped one below 1e-13 of
// sum_e |V_e| at the window's edge).

// Edge-weight moments of one (64-row tile, chunk): lane = row, the chunk's
// edges e0[c] .. e0[c + 1] in order (edge records and tables wave-uniform).
// what = 0: the K block moments of W for the blocks the chunk emits, into mom
// [K][n_blk][rows] (rows fastest, so the stores of a wave are contiguous), or
// for a block the plan cuts, the chunk's piece into part [slot][K][rows];
// what = 1: S_m, m0 <= m < m0 + K (m < mh), over the
// chunk's edges into hpart [chunk][rows][mh]; chunk 0 also writes the
// constant norm part hhc [rows].
template <int ND, int PREC, int K, int WHAT>
__global__ void __launch_bounds__(64) k_het_tmom(const double* __restrict__ coef, int64_t ld, int64_t n,
                                                 const double* __restrict__ rec, int n_bins,
                                                 const double* __restrict__ tab, int mh,
                                                 const int32_t* __restrict__ bs, const int32_t* __restrict__ plan,
                                                 int nch, int n_blk, int m0, HetConst hc, TrigConsts T,
                                                 double2* __restrict__ mom, double2* __restrict__ part,
                                                 double2* __restrict__ hpart, double* __restrict__ hhc) {
  constexpr int RS = het_rs(ND);
  constexpr int BO = het_bin_off(ND);
  const int64_t p = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t pc = p < n ? p : n - 1;
  const int ch = blockIdx.y;
  const double* cf = coef + pc;
  PhaseCoef c;
  c.a0 = cf[C_A0 * ld]; c.a2 = cf[C_A2 * ld]; c.a3 = cf[C_A3 * ld]; c.a4 = cf[C_A4 * ld];
  c.a5 = cf[C_A5 * ld]; c.a6 = cf[C_A6 * ld]; c.a7 = cf[C_A7 * ld]; c.a8 = cf[C_A8 * ld];
  c.a10 = cf[C_A10 * ld]; c.a12 = cf[C_A12 * ld]; c.b5 = cf[C_B5 * ld]; c.b6 = cf[C_B6 * ld];
  double dt[ND], qr[ND], qi[ND], q2[ND], pr[ND], pim[ND];
  double hconst = 0.0;
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    dt[i] = i == 0 ? 0.0 : cf[(C_DT1 + i - 1) * ld];
    const double ar = cf[(C_APRE + i) * ld], ai = cf[(C_APIM + i) * ld];
    qr[i] = ar * hc.ap0_inv_re[i] - ai * hc.ap0_inv_im[i];
    qi[i] = ar * hc.ap0_inv_im[i] + ai * hc.ap0_inv_re[i];
    q2[i] = qr[i] * qr[i] + qi[i] * qi[i];
    hconst = fma(q2[i], hc.hh0[i], hconst);
    pr[i] = pim[i] = 0.0;
  }
  if (WHAT == 0 && ch == 0 && p < n) hhc[p] = hconst;
  const int32_t* __restrict__ e0 = plan;
  const int e_lo = e0[ch], e_hi = e0[ch + 1];
  const int tw_ = K + mh;  // table row length
  if (WHAT == 1 && e_lo > 0) {  // the norm term needs the previous edge's phasors
    const double* r = rec + (int64_t)(e_lo - 1) * RS;
    const double d0 = phase_cycles(c, r[H_X], r[H_X2], r[H_XM5], r[H_LNF]) - r[H_PHI0];
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const double di = i == 0 ? d0 : fma(r[H_F], dt[i], d0) - r[H_PHI0 + i];
      het_phasor<PREC>(di, T, &pr[i], &pim[i]);
    }
  }
  double ar_[K], ai_[K];
#pragma unroll
  for (int m = 0; m < K; ++m) ar_[m] = ai_[m] = 0.0;
  // one edge: its weight (W_e for WHAT = 0, V_e for WHAT = 1) into the moments
  auto edge = [&](int e) {
    const double* r = rec + (int64_t)e * RS;
    const double d0 = phase_cycles(c, r[H_X], r[H_X2], r[H_XM5], r[H_LNF]) - r[H_PHI0];
    const double f = r[H_F];
    double wr = 0.0, wi = 0.0;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const double di = i == 0 ? d0 : fma(f, dt[i], d0) - r[H_PHI0 + i];
      double gr, gi;
      het_phasor<PREC>(di, T, &gr, &gi);
      const double* w = r + BO + 1 + 6 * i;
      if constexpr (WHAT == 0) {
        // summed-by-parts weights; the first and last edges take one side
        const double kr = e == 0 ? w[0] - w[2] : (e == n_bins ? w[2] : w[0]);
        const double ki = e == 0 ? w[1] - w[3] : (e == n_bins ? w[3] : w[1]);
        const double kgr = kr * gr - ki * gi, kgi = kr * gi + ki * gr;  // q K g
        wr = fma(qr[i], kgr, fma(-qi[i], kgi, wr));
        wi = fma(qr[i], kgi, fma(qi[i], kgr, wi));
      } else {
        const double sq = e > 0 ? q2[i] * w[4] : 0.0;  // |q|^2 (B0 / 2) g_e conj(g_e-1)
        wr = fma(sq, fma(gr, pr[i], gi * pim[i]), wr);
        wi = fma(sq, fma(gi, pr[i], -gr * pim[i]), wi);
        pr[i] = gr;
        pim[i] = gi;
      }
    }
    const double* tp = tab + (int64_t)e * tw_ + (WHAT == 0 ? 0 : K + m0);
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const double t = (WHAT == 0 || m0 + m < mh) ? tp[m] : 0.0;
      ar_[m] = fma(t, wr, ar_[m]);
      ai_[m] = fma(t, wi, ai_[m]);
    }
  };
  if constexpr (WHAT == 0) {
    const int32_t* __restrict__ blo = e0 + nch + 1;
    const int32_t* __restrict__ bhi = blo + nch;
    const int32_t* __restrict__ sfirst = bhi + nch;
    const int32_t* __restrict__ slast = sfirst + nch;
    const int b_lo = blo[ch], b_hi = bhi[ch];
    int e = e_lo;
    for (int b = b_lo; b < b_hi; ++b) {
      const int be = bs[b + 1] < e_hi ? bs[b + 1] : e_hi;
      for (; e < be; ++e) edge(e);
      const int slot = b == b_hi - 1 ? slast[ch] : (b == b_lo ? sfirst[ch] : -1);
      if (p < n) {  // rows fastest: a wave's 64 rows store 1 KB contiguously
        double2* out = slot < 0 ? mom + (int64_t)b * n + p : part + (int64_t)slot * K * n + p;
        const int64_t ms = slot < 0 ? (int64_t)n_blk * n : n;
#pragma unroll
        for (int m = 0; m < K; ++m) out[m * ms] = make_double2(ar_[m], ai_[m]);
      }
#pragma unroll
      for (int m = 0; m < K; ++m) ar_[m] = ai_[m] = 0.0;
    }
  } else {
    for (int e = e_lo; e < e_hi; ++e) edge(e);
    if (p < n) {
      double2* out = hpart + ((int64_t)ch * n + p) * mh + m0;
#pragma unroll
      for (int m = 0; m < K; ++m)
        if (m0 + m < mh) out[m] = make_double2(ar_[m], ai_[m]);
    }
  }
}

// Blocks the plan cuts: each sums its pieces part [slot][K][rows] in chunk
// order into mom [K][n_blk][rows]; lane = row, one (cut block, order) per
// grid row and layer (a block of the narrow windows' wide blocks can have
// tens of pieces, so the orders run in parallel).
template <int K>
__global__ void __launch_bounds__(64) k_het_tmom_fix(int64_t n, int n_blk, const int32_t* __restrict__ fb,
                                                     const int32_t* __restrict__ fs, const int32_t* __restrict__ fc,
                                                     const double2* __restrict__ part, double2* __restrict__ mom) {
  const int64_t p = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (p >= n) return;
  const int i = blockIdx.y, m = blockIdx.z;
  const int b = fb[i], s0 = fs[i], cnt = fc[i];
  double2 v = part[((int64_t)s0 * K + m) * n + p];
  for (int k = 1; k < cnt; ++k) v = c_add(v, part[((int64_t)(s0 + k) * K + m) * n + p]);
  mom[((int64_t)m * n_blk + b) * n + p] = v;
}

template <int ND, int K>
static void launch_het_tmom_k(gw_ctx* ctx, const double* coef, int64_t ld, int64_t n, int prec, const HetConst& hc,
                              int what, int m0, double2* mom, double2* part, double2* hpart, double* hhc,
                              hipStream_t st) {
  const gw_het_state* h = ctx->het;
  const TrigConsts T = make_trig_consts();
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)h->tm_nch);
  const int32_t* bs = h->tm_idx;
  const int32_t* plan = h->tm_idx + h->tm_nblk + 1;
#define GW_HET_TMOM(P, W)                                                                                     \
  hipLaunchKernelGGL((k_het_tmom<ND, P, K, W>), grid, dim3(64), 0, st, coef, ld, n, (const double*)h->rec,        \
                     h->n_bins, (const double*)h->tm_tab, h->tm_mh, bs, plan, h->tm_nch, h->tm_nblk, m0, hc, T, mom, \
                     part, hpart, hhc)
  if (prec == GW_PREC_FP64) {
    if (what == 0) GW_HET_TMOM(0, 0); else GW_HET_TMOM(0, 1);
  } else {
    if (what == 0) GW_HET_TMOM(1, 0); else GW_HET_TMOM(1, 1);
  }
#undef GW_HET_TMOM
  if (what == 0 && h->tm_nsplit > 0) {  // add the pieces of the cut blocks
    const int32_t* fb = plan + (h->tm_nch + 1) + 4 * h->tm_nch;
    hipLaunchKernelGGL((k_het_tmom_fix<K>), dim3((unsigned)((n + 63) / 64), (unsigned)h->tm_nsplit, K), dim3(64), 0,
                       st, n, h->tm_nblk, fb, fb + h->tm_nsplit, fb + 2 * h->tm_nsplit, (const double2*)part, mom);
  }
}

template <int ND>
static void launch_het_tmom_nd(gw_ctx* ctx, const double* coef, int64_t ld, int64_t n, int prec, const HetConst& hc,
                               int what, int m0, double2* mom, double2* part, double2* hpart, double* hhc,
                               hipStream_t st) {
  if (ctx->het->tm_K == 12)
    launch_het_tmom_k<ND, 12>(ctx, coef, ld, n, prec, hc, what, m0, mom, part, hpart, hhc, st);
  else
    launch_het_tmom_k<ND, 16>(ctx, coef, ld, n, prec, hc, what, m0, mom, part, hpart, hhc, st);
}

// Chunks of the moment kernel: edge ranges of about equal cost (an edge or
// a block's moment stores count one unit each; gw_hetplan.h), the count
// chosen for about 4096 (tile, chunk) waves (at most 256 chunks, each of at
// least 8 units), or fixed by gw_set_het_tm_split.
static int het_tm_chunks(const gw_ctx* ctx, int64_t n, int n_blk) {
  if (ctx->tm_nsk > 0) return ctx->tm_nsk;
  const int64_t tiles = (n + 63) / 64;
  int64_t want = (4096 + tiles - 1) / tiles;
  const int64_t most = std::max<int64_t>(1, std::min<int64_t>(256, (ctx->het->n_edges + n_blk) / 8));
  return (int)std::max<int64_t>(1, std::min(want, most));
}

// Row-independent tables of the time marginal for the grid (blocks of blk
// fine bins, n_blk of them, the window's largest |u| = umax fine-grid cycles)
// and nch edge chunks.
static gw_status het_tm_tables(gw_ctx* ctx, int blk, int n_blk, double umax, int nch, int K) {
  gw_het_state* h = ctx->het;
  if (h->tm_tab && h->tm_blk == blk && h->tm_nblk == n_blk && h->tm_nch_req == nch && h->tm_umax == umax &&
      h->tm_K == K)
    return GW_OK;
  const int ne = h->n_edges;
  std::vector<int64_t> k(ne);
  for (int e = 0; e < ne; ++e) k[e] = (int64_t)llround(h->f_edges[e] / ctx->geom.df) - ctx->geom.k0;
  int64_t dmin = INT64_MAX, dmax = 0;
  for (int e = 1; e < ne; ++e) {
    dmin = std::min(dmin, k[e] - k[e - 1]);
    dmax = std::max(dmax, k[e] - k[e - 1]);
  }
  if (ne < 2) dmin = dmax = 0;
  const double cw = 0.5 * (double)(dmin + dmax), hw = 0.5 * (double)(dmax - dmin);
  // norm series length: (x^M / M!) e^x below 1e-13, x = 2 pi hw umax
  const double x = 2.0 * kPi * hw * umax;
  int mh = 1;
  double term = x;
  while (term * exp(x) > 1e-13 && mh < kTgHMax) {
    ++mh;
    term *= x / (double)mh;
  }
  if (term * exp(x) > 1e-13)
    return set_error(GW_ENOTSUP, "heterodyned time marginal: bin widths up to %lld fine bins over a +-%.3g s window "
                                 "need more than %d norm terms", (long long)dmax, ctx->tm_window, kTgHMax);
  const int tw_ = K + mh;
  std::vector<double> tab((size_t)ne * tw_, 0.0);
  std::vector<int32_t> bs(n_blk + 1, 0);
  const double cen = 0.5 * (blk - 1), hinv = 2.0 / blk;
  for (int e = 0; e < ne; ++e) {
    const int64_t b = k[e] / blk;
    if (b < 0 || b >= n_blk) return set_error(GW_EINVAL, "heterodyned time marginal: edge outside the band");
    bs[b + 1] += 1;
    const double sv = ((double)(k[e] - b * blk) - cen) * hinv;
    tgrid_basis_at(sv, K, tab.data() + (size_t)e * tw_);
    const double sg = e > 0 && hw > 0.0 ? ((double)(k[e] - k[e - 1]) - cw) / hw : 0.0;
    double tp = 1.0;
    for (int m = 0; m < mh; ++m) {
      tab[(size_t)e * tw_ + K + m] = tp;
      tp *= sg;
    }
  }
  for (int b = 0; b < n_blk; ++b) bs[b + 1] += bs[b];
  const HetTmPlan plan = het_tm_plan(bs, n_blk, ne, nch);
  std::vector<int32_t> idx(bs);
  for (const std::vector<int32_t>* v : {&plan.e0, &plan.blo, &plan.bhi, &plan.sfirst, &plan.slast, &plan.fb,
                                        &plan.fs, &plan.fc})
    idx.insert(idx.end(), v->begin(), v->end());
  if (h->tm_tab) (void)hipFree(h->tm_tab);
  if (h->tm_idx) (void)hipFree(h->tm_idx);
  h->tm_tab = nullptr;
  h->tm_idx = nullptr;
  gw_status s = check_hip(hipMalloc((void**)&h->tm_tab, tab.size() * sizeof(double)), "time-marginal tables");
  if (s == GW_OK) s = check_hip(hipMalloc((void**)&h->tm_idx, idx.size() * sizeof(int32_t)), "time-marginal index");
  if (s == GW_OK)
    s = check_hip(hipMemcpy(h->tm_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice), "tables");
  if (s == GW_OK)
    s = check_hip(hipMemcpy(h->tm_idx, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice), "index");
  if (s != GW_OK) return s;
  h->tm_blk = blk;
  h->tm_nblk = n_blk;
  h->tm_mh = mh;
  h->tm_nch = plan.nch();
  h->tm_nch_req = nch;
  h->tm_nslot = plan.nslot;
  h->tm_nsplit = (int)plan.fb.size();
  h->tm_hw = hw;
  h->tm_c2 = dmin + dmax;
  h->tm_umax = umax;
  h->tm_K = K;
  return GW_OK;
}

gw_status loglike_het_tmarg(gw_ctx* ctx, const double* theta, int64_t n, int prec, double* logl, hipStream_t st) {
  return loglike_het_tmarg_staged(ctx, theta, n, prec, logl, nullptr, st);
}

gw_status loglike_het_tmarg_staged(gw_ctx* ctx, const double* theta, int64_t n, int prec, double* logl, double* zout,
                                   hipStream_t st) {
  gw_het_state* h = ctx->het;
  if (!h) return set_error(GW_ESTATE, "loglike_batch: heterodyne_setup has not been called");
  TimeGridShape g;
  gw_status s = time_grid_shape(ctx, &g);
  const int K = tgrid_orders(g.L, g.jmax);
  if (s == GW_OK) s = tgrid_tables(ctx, g.L, g.jmax, K);
  const int64_t chunk = tgrid_chunk_rows(n, g.n_blk, K);
  // edge chunks sized for the rows of one launch
  const int nch = het_tm_chunks(ctx, chunk, g.n_blk);
  const double umax = (double)g.jmax / ((double)g.N * (double)g.R);
  if (s == GW_OK) s = het_tm_tables(ctx, g.blk, g.n_blk, umax, nch, K);
  if (s != GW_OK) return s;
  const int mh = h->tm_mh;
  // workspace: coefficients for all rows; per row chunk the moments
  // [K][n_blk][rows] (rows fastest), the pieces of cut blocks [slot][K][rows],
  // the norm moments [n_ch][rows][mh], hhc [rows] and, for a small launch,
  // the order groups' partial grids (16-byte aligned)
  const int64_t zp = tgrid_zpart_elems(n, chunk, K, 2 * g.jmax + 1);
  s = ensure_buffer(&ctx->coef, &ctx->coef_cap, (int64_t)C_NCOEF * n, "coefficient workspace");
  if (s == GW_OK)
    s = ensure_buffer(&ctx->tm_mom, &ctx->tm_mom_cap,
                      chunk * K * g.n_blk * 2 + (int64_t)h->tm_nslot * K * chunk * 2 +
                          (int64_t)h->tm_nch * chunk * mh * 2 + chunk + 1 + 2 * zp,
                      "time-marginal workspace");
  if (s != GW_OK || !theta) return s;  // theta NULL: reserve only
  double2* mom = (double2*)ctx->tm_mom;
  double2* part = mom + chunk * K * g.n_blk;
  double2* hpart = part + (int64_t)h->tm_nslot * K * chunk;
  double* hhc = (double*)(hpart + (int64_t)h->tm_nch * chunk * mh);
  double* zpart = zp > 0 ? hhc + (chunk + 1) / 2 * 2 : nullptr;
  s = launch_prologue(ctx, theta, n, GW_MARG_PHASE_TIME, ctx->coef, n, st);
  if (s != GW_OK) return s;
  HetConst hc;
  for (int i = 0; i < kMaxDet; ++i) {
    hc.ap0_inv_re[i] = h->ap0_inv_re[i];
    hc.ap0_inv_im[i] = h->ap0_inv_im[i];
    hc.hh0[i] = h->hh0[i];
  }
  hc.dd = ctx->dd;
  const int nt = 2 * g.jmax + 1;
  for (int64_t r0 = 0; r0 < n && s == GW_OK; r0 += chunk) {
    const int64_t cn = n - r0 < chunk ? n - r0 : chunk;
    const int prof = prof_begin(ctx, st, 1);
    for (int what = 0; what < 2; ++what)
      for (int m0 = 0; m0 < (what == 0 ? 1 : mh); m0 += K) {
        switch (ctx->n_det) {
          case 1:
            launch_het_tmom_nd<1>(ctx, ctx->coef + r0, n, cn, prec, hc, what, m0, mom, part, hpart, hhc, st);
            break;
          case 2:
            launch_het_tmom_nd<2>(ctx, ctx->coef + r0, n, cn, prec, hc, what, m0, mom, part, hpart, hhc, st);
            break;
          case 3:
            launch_het_tmom_nd<3>(ctx, ctx->coef + r0, n, cn, prec, hc, what, m0, mom, part, hpart, hhc, st);
            break;
          case 4:
            launch_het_tmom_nd<4>(ctx, ctx->coef + r0, n, cn, prec, hc, what, m0, mom, part, hpart, hhc, st);
            break;
          default: return set_error(GW_ENOTSUP, "n_det not supported");
        }
        s = check_hip(hipGetLastError(), "time-marginal moment launch");
        if (s != GW_OK) return s;
      }
    prof_end(ctx, prof, st);
    TGridArgs a{};
    a.mom = (const double*)mom;
    a.mom_rs = 1;  // k_het_tmom writes rows fastest
    a.mom_es = cn;
    a.n = cn;
    a.n_blk = g.n_blk;
    a.L = g.L;
    a.jmax = g.jmax;
    a.K = K;
    a.coef = ctx->coef + r0;
    a.ld = n;
    a.logl = logl + r0;
    a.het = 1;
    a.hhc = hhc;
    a.hpart = (const double*)hpart;
    a.n_hch = h->tm_nch;
    a.mh = mh;
    a.hw_step = 2.0 * kPi * h->tm_hw / ((double)g.N * (double)g.R);
    a.c2 = h->tm_c2;
    a.cden = 2 * g.N * (int64_t)g.R;
    a.zout = zout ? zout + r0 * nt * 3 : nullptr;
    a.f0_num = (double)(2 * ctx->geom.k0 + g.blk - 1);
    a.f0_den = (double)(2 * g.N) * (double)g.R;
    a.zpart = zpart;
    const int gslot = prof_begin(ctx, st, 2);
    s = launch_tgrid(ctx, a, st);
    prof_end(ctx, gslot, st);
  }
  return s;
}

gw_status loglike_het(gw_ctx* ctx, const double* theta, int64_t n, int marg, int prec, double* logl, hipStream_t st) {
  if (!ctx->het) return set_error(GW_ESTATE, "loglike_batch: heterodyne_setup has not been called");
  if (marg == GW_MARG_PHASE_TIME) return loglike_het_tmarg(ctx, theta, n, prec, logl, st);
  return loglike_het_staged(ctx, theta, n, marg, prec, logl, nullptr, st);
}

gw_status loglike_het_staged(gw_ctx* ctx, const double* theta, int64_t n, int marg, int prec, double* logl,
                             double* zc3, hipStream_t st) {
  if (!ctx->het) return set_error(GW_ESTATE, "heterodyne_setup has not been called");
  int n_ech = 1;
  gw_status s = het_prepare(ctx, theta, nullptr, 1, n, logl, true, &n_ech, st, zc3);
  if (s != GW_OK) return s;
  return enqueue_het(ctx, marg, prec, n_ech, st);
}

}  // namespace gw

using namespace gw;

extern "C" {

gw_status heterodyne_setup(gw_ctx* ctx, const double* theta0, int32_t n_bins, int32_t bin_rule, double* edges_out) {
  if (!ctx) return set_error(GW_EINVAL, "heterodyne_setup: ctx is NULL");
  if (!theta0) return set_error(GW_EINVAL, "heterodyne_setup: theta0 is NULL");
  if (bin_rule != 0 && bin_rule != 1) return set_error(GW_EINVAL, "heterodyne_setup: bin_rule must be 0 or 1");
  if (n_bins < 1 || (int64_t)n_bins > ctx->geom.n_freq - 1)
    return set_error(GW_EINVAL, "heterodyne_setup: n_bins must be in 1 .. n_freq - 1");
  for (int j = 0; j < 13; ++j)
    if (!isfinite(theta0[j])) return set_error(GW_EINVAL, "heterodyne_setup: theta0 must be finite");
  if (!(theta0[0] > 0.0) || !(theta0[1] > 0.0) || theta0[1] > 1.0 || fabs(theta0[2]) >= 1.0 ||
      fabs(theta0[3]) >= 1.0 || !(theta0[6] > 0.0))
    return set_error(GW_EINVAL, "heterodyne_setup: theta0 is unphysical");
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  het_free(ctx);
  if (ctx->graphs) graphs_clear(ctx->graphs);

  const int nd = ctx->n_det;
  const int64_t nf = ctx->geom.n_freq;
  std::vector<int64_t> edges = make_edges(ctx->geom, n_bins, bin_rule);
  const int ne = (int)edges.size();
  gw_het_state* h = new (std::nothrow) gw_het_state();
  if (!h) return set_error(GW_ENOMEM, "heterodyne_setup: host allocation");
  h->n_edges = ne;
  h->n_bins = ne - 1;
  h->rs = het_rs(nd);
  h->theta0.assign(theta0, theta0 + 13);
  h->max_sub = kMaxSub;
  h->f_edges.resize(ne);
  for (int e = 0; e < ne; ++e) h->f_edges[e] = (double)(ctx->geom.k0 + edges[e]) * ctx->geom.df;

  // hh weights 4 df f^(-7/3) / S for the set-up sums
  std::vector<double> hw((size_t)nd * nf);
  for (int i = 0; i < nd; ++i)
    for (int64_t k = 0; k < nf; ++k) {
      const double f = (double)(ctx->geom.k0 + k) * ctx->geom.df;
      hw[(size_t)i * nf + k] = 4.0 * ctx->geom.df * pow(f, -7.0 / 3.0) / ctx->h_psd[(size_t)i * nf + k];
    }
  double *d_hw = nullptr, *d_th = nullptr, *d_coef0 = nullptr;
  int64_t* d_edges = nullptr;
  auto cleanup = [&]() {
    if (d_hw) (void)hipFree(d_hw);
    if (d_th) (void)hipFree(d_th);
    if (d_coef0) (void)hipFree(d_coef0);
    if (d_edges) (void)hipFree(d_edges);
  };
  s = check_hip(hipMalloc((void**)&d_hw, hw.size() * sizeof(double)), "het alloc");
  if (s == GW_OK) s = check_hip(hipMalloc((void**)&d_th, 13 * sizeof(double)), "het alloc");
  if (s == GW_OK) s = check_hip(hipMalloc((void**)&d_coef0, C_NCOEF * sizeof(double)), "het alloc");
  if (s == GW_OK) s = check_hip(hipMalloc((void**)&d_edges, ne * sizeof(int64_t)), "het alloc");
  if (s == GW_OK) s = check_hip(hipMalloc((void**)&h->rec, (size_t)ne * h->rs * sizeof(double)), "het alloc");
  if (s == GW_OK) s = check_hip(hipMalloc((void**)&h->args, sizeof(HetArgs)), "het alloc");
  if (s == GW_OK) s = check_hip(hipMalloc((void**)&h->tile_pre, (kMaxSub + 1) * sizeof(int64_t)), "het alloc");
  if (s == GW_OK) s = check_hip(hipMalloc((void**)&h->subs_single, 2 * sizeof(int64_t)), "het alloc");
  if (s == GW_OK) s = check_hip(hipMemcpy(d_hw, hw.data(), hw.size() * sizeof(double), hipMemcpyHostToDevice), "copy");
  if (s == GW_OK) s = check_hip(hipMemcpy(d_th, theta0, 13 * sizeof(double), hipMemcpyHostToDevice), "copy");
  if (s == GW_OK)
    s = check_hip(hipMemcpy(d_edges, edges.data(), ne * sizeof(int64_t), hipMemcpyHostToDevice), "copy");
  if (s == GW_OK) s = check_hip(hipMemset(h->rec, 0, (size_t)ne * h->rs * sizeof(double)), "memset");
  if (s == GW_OK) s = launch_prologue(ctx, d_th, 1, 0, d_coef0, 1, nullptr);
  const TrigConsts T = make_trig_consts();
  if (s == GW_OK) {
    hipLaunchKernelGGL(k_het_edges, dim3((ne + 255) / 256), dim3(256), 0, nullptr, ctx->bins, ctx->rec_stride,
                       d_edges, ne, nd, d_coef0, T, ctx->geom.k0, ctx->geom.df, h->rec);
    s = check_hip(hipGetLastError(), "het edge kernel");
  }
  if (s == GW_OK) {
    hipLaunchKernelGGL(k_het_summary, dim3(ne - 1, nd), dim3(256), 0, nullptr, ctx->bins, ctx->rec_stride, d_hw, nf,
                       d_edges, ne - 1, d_coef0, T, ctx->geom.k0, ctx->geom.df, h->rec, nd);
    s = check_hip(hipGetLastError(), "het summary kernel");
  }
  double coef0[C_NCOEF];
  if (s == GW_OK) s = check_hip(hipMemcpy(coef0, d_coef0, sizeof(coef0), hipMemcpyDeviceToHost), "copy");
  if (s == GW_OK) s = check_hip(hipDeviceSynchronize(), "heterodyne set-up");
  cleanup();
  if (s != GW_OK) {
    free_state(h);
    return s;
  }
  for (int i = 0; i < nd; ++i) {
    const double ar = coef0[C_APRE + i], ai = coef0[C_APIM + i];
    const double m = ar * ar + ai * ai;
    if (!(m > 0.0)) {
      free_state(h);
      return set_error(GW_EINVAL, "heterodyne_setup: reference template vanishes in detector %d", i);
    }
    h->ap0_inv_re[i] = ar / m;
    h->ap0_inv_im[i] = -ai / m;
  }
  // Bin summaries -> per-edge weights of the summed-by-parts sums.
  {
    const int rs = h->rs, bo = het_bin_off(nd), nb = ne - 1;
    std::vector<double> rh((size_t)ne * rs);
    s = check_hip(hipMemcpy(rh.data(), h->rec, rh.size() * sizeof(double), hipMemcpyDeviceToHost), "copy");
    if (s != GW_OK) {
      free_state(h);
      return s;
    }
    std::vector<double> out(rh);
    for (int i = 0; i < nd; ++i) {
      double hh0 = 0.0;
      for (int e = 0; e < ne; ++e) {
        double rr = 0.0, ri = 0.0, lr = 0.0, li = 0.0, b0h = 0.0;
        if (e >= 1) {  // bin e: right edge e
          const double* sb = &rh[(size_t)e * rs + bo + 1 + 6 * i];
          const double inv = rh[(size_t)e * rs + bo];
          rr = 0.5 * sb[0] + sb[2] * inv;
          ri = 0.5 * sb[1] + sb[3] * inv;
          b0h = 0.5 * sb[4];
          hh0 += b0h;
        }
        if (e + 1 <= nb) {  // bin e + 1: left edge e
          const double* sb = &rh[(size_t)(e + 1) * rs + bo + 1 + 6 * i];
          const double inv = rh[(size_t)(e + 1) * rs + bo];
          lr = 0.5 * sb[0] - sb[2] * inv;
          li = 0.5 * sb[1] - sb[3] * inv;
        }
        double* o = &out[(size_t)e * rs + bo + 1 + 6 * i];
        o[0] = rr + lr;
        o[1] = ri + li;
        o[2] = rr;
        o[3] = ri;
        o[4] = b0h;
        o[5] = 0.0;
      }
      h->hh0[i] = hh0;
    }
    s = check_hip(hipMemcpy(h->rec, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice), "copy");
    if (s != GW_OK) {
      free_state(h);
      return s;
    }
  }
  ctx->het = h;
  ++ctx->gen;
  if (edges_out)
    for (int e = 0; e < ne; ++e) edges_out[e] = h->f_edges[e];
  return GW_OK;
}

gw_status gw_het_info(const gw_ctx* ctx, int32_t* n_bins) {
  if (!ctx || !n_bins) return set_error(GW_EINVAL, "gw_het_info: null argument");
  if (!ctx->het) return set_error(GW_ESTATE, "gw_het_info: heterodyne_setup has not been called");
  *n_bins = ctx->het->n_bins;
  return GW_OK;
}

gw_status loglike_batch_uneven(gw_ctx* ctx, const double* theta, int64_t n_rows, const int64_t* subs, int32_t n_sub,
                               int32_t like, int32_t marg, int32_t prec, int32_t use_graph, double* logl,
                               void* stream) {
  if (!ctx) return set_error(GW_EINVAL, "loglike_batch_uneven: ctx is NULL");
  if (n_rows < 0 || n_sub < 0) return set_error(GW_EINVAL, "loglike_batch_uneven: negative size");
  if (n_sub > kMaxSub) return set_error(GW_EINVAL, "loglike_batch_uneven: at most %d sub-batches", kMaxSub);
  if (n_sub > 0 && (!theta || !subs || !logl)) return set_error(GW_EINVAL, "loglike_batch_uneven: null pointer");
  if (like != GW_HET) return set_error(GW_ENOTSUP, "loglike_batch_uneven: only GW_HET is supported");
  if (marg < GW_MARG_NONE || marg > GW_MARG_PHASE_DIST) return set_error(GW_EINVAL, "loglike_batch_uneven: bad marg");
  if (prec != GW_PREC_FP64 && prec != GW_PREC_MIXED) return set_error(GW_EINVAL, "loglike_batch_uneven: bad prec");
  if (marg == GW_MARG_PHASE_DIST && ctx->n_dist <= 0)
    return set_error(GW_ESTATE, "loglike_batch_uneven: distance marginal needs a distance grid");
  if (!ctx->het) return set_error(GW_ESTATE, "loglike_batch_uneven: heterodyne_setup has not been called");
  if (n_sub == 0 || n_rows == 0) return GW_OK;
  hipStream_t st = (hipStream_t)stream;
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  gw_het_state* h = ctx->het;
  int n_ech = 1;
  s = het_prepare(ctx, theta, subs, n_sub, n_rows, logl, false, &n_ech, st);
  if (s != GW_OK) return s;
  if (!use_graph || ctx->prof) return enqueue_het(ctx, marg, prec, n_ech, st);

  if (!ctx->graphs) {
    ctx->graphs = new (std::nothrow) gw_graph_cache();
    if (!ctx->graphs) return set_error(GW_ENOMEM, "graph cache");
  }
  gw_graph_cache* gc = ctx->graphs;
  const GraphKey key{marg, prec, h->wpb, h->grid, n_ech, h->n_rows_last >= kDistRowsPerLane ? 1 : 0};
  auto it = gc->exec.find(key);
  if (it == gc->exec.end()) {
    if (!gc->cap_stream) {
      s = check_hip(hipStreamCreateWithFlags(&gc->cap_stream, hipStreamNonBlocking), "capture stream");
      if (s != GW_OK) return s;
    }
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    s = check_hip(hipStreamBeginCapture(gc->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    if (s != GW_OK) return s;
    gw_status sq = enqueue_het(ctx, marg, prec, n_ech, gc->cap_stream);
    s = check_hip(hipStreamEndCapture(gc->cap_stream, &g), "end capture");
    if (sq != GW_OK) {
      if (g) (void)hipGraphDestroy(g);
      return sq;
    }
    if (s != GW_OK) return s;
    const auto t0 = std::chrono::steady_clock::now();
    s = check_hip(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0), "graph instantiate");
    const auto t1 = std::chrono::steady_clock::now();
    gc->last_instantiate_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (s != GW_OK) {
      (void)hipGraphDestroy(g);
      return s;
    }
    gc->graph[key] = g;
    gc->exec[key] = ge;
    it = gc->exec.find(key);
  }
  return check_hip(hipGraphLaunch(it->second, st), "graph launch");
}

gw_status gw_set_het_shape(gw_ctx* ctx, int32_t waves_per_block, int32_t grid, int32_t n_ech) {
  if (!ctx) return set_error(GW_EINVAL, "gw_set_het_shape: ctx is NULL");
  if (!ctx->het) return set_error(GW_ESTATE, "gw_set_het_shape: heterodyne_setup has not been called");
  if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
    return set_error(GW_EINVAL, "gw_set_het_shape: waves_per_block must be 1, 2 or 4");
  if (grid < 0 || grid > (1 << 20)) return set_error(GW_EINVAL, "gw_set_het_shape: grid out of range");
  if (n_ech < 0 || n_ech > 256) return set_error(GW_EINVAL, "gw_set_het_shape: n_ech must be 0 .. 256");
  ctx->het->wpb = waves_per_block;
  ctx->het->grid = grid;
  ctx->het->ech = n_ech;
  ++ctx->gen;
  return GW_OK;
}

gw_status gw_set_het_tm_split(gw_ctx* ctx, int32_t n_chunks) {
  if (!ctx) return set_error(GW_EINVAL, "gw_set_het_tm_split: ctx is NULL");
  if (n_chunks < 0 || n_chunks > 256 || (n_chunks & (n_chunks - 1)) != 0)
    return set_error(GW_EINVAL, "gw_set_het_tm_split: n_chunks must be 0 or a power of two up to 256");
  ctx->tm_nsk = n_chunks;
  ++ctx->gen;
  return GW_OK;
}

gw_status gw_graph_info(const gw_ctx* ctx, int32_t* n_graphs, double* last_instantiate_ms) {
  if (!ctx || !n_graphs || !last_instantiate_ms) return set_error(GW_EINVAL, "gw_graph_info: null argument");
  *n_graphs = ctx->graphs ? (int32_t)ctx->graphs->exec.size() : 0;
  *last_instantiate_ms = ctx->graphs ? ctx->graphs->last_instantiate_ms : 0.0;
  return GW_OK;
}

// Autotuner: time every candidate launch shape on the caller's batch and keep
// the fastest in the context.  Candidates: full band, proposals per workgroup
// {64, 128, 256} x frequency chunks {8 .. 512} (multiples of 8, at least 16
// bins per chunk); heterodyned, waves per workgroup {1, 2, 4} x persistent
// grid {8, 16, 32, 64} waves per CU x edge chunks {heuristic, 8, 16, 32}.
gw_status gw_autotune(gw_ctx* ctx, const double* theta, int64_t n, int32_t like, int32_t marg, int32_t prec,
                      int32_t reps, int32_t* best_shape, double* best_ms, void* stream) {
  if (!ctx || !theta || !best_shape || !best_ms) return set_error(GW_EINVAL, "gw_autotune: null argument");
  if (n < 1 || reps < 1) return set_error(GW_EINVAL, "gw_autotune: n and reps must be >= 1");
  if (like != GW_FULL && like != GW_HET) return set_error(GW_EINVAL, "gw_autotune: bad like");
  if (like == GW_HET && !ctx->het) return set_error(GW_ESTATE, "gw_autotune: heterodyne_setup has not been called");
  hipStream_t st = (hipStream_t)stream;
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  double* out = nullptr;
  s = check_hip(hipMalloc((void**)&out, (size_t)n * sizeof(double)), "autotune output");
  if (s != GW_OK) return s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const bool prof = ctx->prof;
  ctx->prof = false;
  struct Cand {
    int a, b, c;
  };
  std::vector<Cand> cands;
  if (like == GW_FULL) {
    for (int tpb : {64, 128, 256})
      for (int ch : {8, 16, 32, 64, 128, 256, 512})
        if (ctx->geom.n_freq / ch >= 16) cands.push_back({tpb, ch, 0});
  } else {
    for (int w : {1, 2, 4})
      for (int per_cu : {8, 16, 32, 64})
        for (int ech : {0, 8, 16, 32}) cands.push_back({w, 256 * per_cu, ech});
  }
  double best = 1e300;
  Cand arg{0, 0, 0};
  for (const Cand& cand : cands) {
    if (like == GW_FULL) {
      ctx->full_tpb = cand.a;
      ctx->full_chunks = cand.b;
    } else {
      ctx->het->wpb = cand.a;
      ctx->het->grid = cand.b / cand.a;
      ctx->het->ech = cand.c;
    }
    s = loglike_batch(ctx, theta, n, like, marg, prec, out, st);  // warm-up
    if (s != GW_OK) break;
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps && s == GW_OK; ++r) s = loglike_batch(ctx, theta, n, like, marg, prec, out, st);
    (void)hipEventRecord(e1, st);
    if (s != GW_OK) break;
    s = check_hip(hipEventSynchronize(e1), "autotune sync");
    if (s != GW_OK) break;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double per = ms / reps;
    if (per < best) {
      best = per;
      arg = cand;
    }
  }
  if (like == GW_FULL) {
    ctx->full_tpb = arg.a;
    ctx->full_chunks = arg.b;
  } else {
    ctx->het->wpb = arg.a > 0 ? arg.a : 4;
    ctx->het->grid = arg.a > 0 ? arg.b / arg.a : 0;
    ctx->het->ech = arg.c;
    if (ctx->graphs) graphs_clear(ctx->graphs);
  }
  ctx->prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (s != GW_OK) return s;
  best_shape[0] = arg.a;
  best_shape[1] = like == GW_FULL ? arg.b : ctx->het->grid;
  best_shape[2] = arg.c;
  *best_ms = best;
  return GW_OK;
}

}  // extern "C"
