// Full-band batched likelihood: per-proposal prologue, the fused
// phase/phasor/projection/overlap kernel and the FP64 epilogue with the
// phase and distance marginalisations (Sec. III.A).
//
// Layout.  One lane owns one proposal; a workgroup owns ``tpb`` proposals
// (one to four waves) and one contiguous chunk of frequency bins, which all
// of its waves walk in step so that they share each bin record.  Every lane of a wave walks the same
// bins in the same order, so the per-bin records (frequency powers and the
// weighted data u_ik = 4 df d_ik* f^(-7/6) / S_ik) are wave-uniform and are
// fetched with scalar loads into SGPRs; the proposal's phase coefficients live
// in VGPRs.  Per bin a lane evaluates the TaylorF2 phase in FP64 (Horner in
// x = f^(1/3); the mixed form only on the first bins of each run and by a
// cubic recurrence in between, see PhaseRuns), one complex phasor
// exp(-i Phi_0) for detector 0, and folds the
// other detectors' linear time-shift phases into a Horner recurrence over the
// bins of the chunk: S_i <- S_i rho_i + u_ik g_k with rho_i = exp(-2 pi i df
// (tau_i - tau_0)), which is multiplied by exp(-2 pi i f_start (tau_i - tau_0))
// at the end.  The template norm <h|h> has a closed form (|h|^2 / S does not
// depend on the phase), so only z_i = sum_k u_ik exp(-i Phi_ik) is summed.
// Partial sums per (chunk, proposal) are combined in a fixed order by the
// epilogue, so results are bitwise reproducible.
#include <math.h>

#include "gw_ctx.h"
#include "gw_phase.h"

namespace gw {

__global__ void __launch_bounds__(256) k_prologue(const double* __restrict__ theta, int64_t n, int marg,
                                                  Geom geom, double* __restrict__ coef, int64_t ld) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  prologue(theta + p * 13, marg, geom, coef + p, ld);
}

// Decode a workgroup index into (chunk, proposal tile).  Workgroups are
// dealt round-robin to the 8 XCDs; when n_chunks is a multiple of 8 all
// workgroups of one chunk land on one XCD so its L2 holds that chunk's bins.
__device__ inline void decode_block(int bid, int nptile, int n_chunks, int* chunk, int* ptile) {
  if ((n_chunks & 7) == 0) {
    const int slot = bid >> 3;
    *chunk = (bid & 7) + 8 * (slot / nptile);
    *ptile = slot % nptile;
  } else {
    *chunk = bid / nptile;
    *ptile = bid % nptile;
  }
}

// Add the sums of waves 1 .. W-1 (W <= 4) of the workgroup to wave 0's, in
// wave order (lane l of every wave holds row l); true on wave 0, which then
// owns them.
template <int ND>
__device__ inline bool wave_sums_combine(double* zr, double* zi) {
  __shared__ double red[3][2 * ND][64];
  const int nw = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (nw == 1) return true;
  if (wv > 0) {
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      red[wv - 1][2 * i][lane] = zr[i];
      red[wv - 1][2 * i + 1][lane] = zi[i];
    }
  }
  __syncthreads();
  if (wv != 0) return false;
  for (int w = 0; w < nw - 1; ++w) {
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      zr[i] += red[w][2 * i][lane];
      zi[i] += red[w][2 * i + 1][lane];
    }
  }
  return true;
}

template <int PREC>
__device__ inline void phasor(double r, const TrigConsts& T, double* gr, double* gi) {
  if (PREC == 0) {
    double s, c;
    sincos_cycles(r, T, &s, &c);
    *gr = c;
    *gi = -s;
  } else {
    // FP64 reduction to a fraction of a cycle, FP32 hardware sin/cos
    // (argument in revolutions).
    const float t = (float)(r - rint(r));
    *gr = (double)__builtin_amdgcn_cosf(t);
    *gi = -(double)__builtin_amdgcn_sinf(t);
  }
}

// LIST (small batches, e.g. the sampler's rounds): the rows are
// rows[0 .. *count) (at most n, in any order) instead of 0 .. n - 1, 64 to a
// workgroup, and the workgroup's waves split the chunk's bins between them
// (each with its own start phase), their sums added in wave order; workgroups
// past the count exit at once.
template <int ND, int PREC, bool LIST>
__global__ void __launch_bounds__(256) k_full(const double* __restrict__ coef, int64_t ld, int64_t n,
                                              const double* __restrict__ bins, int64_t k0, double df,
                                              int n_freq, int chunk_len, int n_chunks, TrigConsts T, PhaseRuns R,
                                              double pg_re, double pg_im, const int32_t* __restrict__ rows,
                                              const int32_t* __restrict__ count, double* __restrict__ partial) {
  constexpr int RS = 4 + 2 * ND;
  const int tpb = LIST ? 64 : blockDim.x;
  const int nptile = (int)((n + tpb - 1) / tpb);
  int chunk, ptile;
  decode_block(blockIdx.x, nptile, n_chunks, &chunk, &ptile);
  int64_t p, pc;
  bool live;
  if constexpr (LIST) {
    const int cnt = *count;
    if (ptile * tpb >= cnt) return;  // uniform over the workgroup
    const int idx = ptile * tpb + (threadIdx.x & 63);
    live = idx < cnt;
    p = rows[live ? idx : cnt - 1];
    pc = p;
  } else {
    p = (int64_t)ptile * tpb + threadIdx.x;
    pc = p < n ? p : n - 1;
    live = p < n;
  }

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

  int kb = chunk * chunk_len;
  int ke = kb + chunk_len < n_freq ? kb + chunk_len : n_freq;
  if constexpr (LIST) {
    // wave index made visibly wave-uniform, so that the bin walk stays scalar
    const int nw = blockDim.x >> 6, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sub = ((ke > kb ? ke - kb : 0) + nw - 1) / nw;
    const int b2 = kb + wv * sub;
    ke = b2 + sub < ke ? b2 + sub : ke;
    kb = b2;
  }

  double zr[ND], zi[ND];
  double rr[ND], ri[ND];  // rho_i
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    zr[i] = 0.0;
    zi[i] = 0.0;
    rr[i] = 1.0;
    ri[i] = 0.0;
  }
#pragma unroll
  for (int i = 1; i < ND; ++i) {
    const double dt = coef[(C_DT1 + i - 1) * ld + pc];
    double s, co;
    sincos_cycles(df * dt, T, &s, &co);
    rr[i] = co;
    ri[i] = -s;
  }

  // Descending walk so that the Horner recurrence leaves rho^0 on the first
  // bin.  Records alternate between two register sets: while one bin is
  // processed the next one's record is already in flight.
  auto accumulate = [&](const double* __restrict__ u, double gr, double gi) {
    {
      const double ur = u[0], ui = u[1];
      zr[0] = fma(ur, gr, zr[0]);
      zr[0] = fma(-ui, gi, zr[0]);
      zi[0] = fma(ur, gi, zi[0]);
      zi[0] = fma(ui, gr, zi[0]);
    }
#pragma unroll
    for (int i = 1; i < ND; ++i) {
      const double ur = u[2 * i], ui = u[2 * i + 1];
      double tr = zr[i] * rr[i];
      tr = fma(-zi[i], ri[i], tr);
      tr = fma(ur, gr, tr);
      tr = fma(-ui, gi, tr);
      double ti = zr[i] * ri[i];
      ti = fma(zi[i], rr[i], ti);
      ti = fma(ur, gi, ti);
      ti = fma(ui, gr, ti);
      zr[i] = tr;
      zi[i] = ti;
    }
  };
  if constexpr (PREC == 0) {
    auto step = [&](const double* __restrict__ rec) {
      const double r = phase_cycles(c, rec[0], rec[1], rec[2], rec[3]);
      double gr, gi;
      phasor<PREC>(r, T, &gr, &gi);
      accumulate(rec + 4, gr, gi);
    };
    if (ke > kb) {
      // bins in pairs with one loop exit (see the mixed form below)
      double ra[RS], rb[RS];
#pragma unroll
      for (int j = 0; j < RS; ++j) ra[j] = bins[(int64_t)(ke - 1) * RS + j];
      int k = ke - 1, left = ke - kb;
      for (; left >= 2; left -= 2, k -= 2) {
#pragma unroll
        for (int j = 0; j < RS; ++j) rb[j] = bins[(int64_t)(k - 1) * RS + j];
        step(ra);
        const int k2 = k - 2 >= kb ? k - 2 : kb;
#pragma unroll
        for (int j = 0; j < RS; ++j) ra[j] = bins[(int64_t)k2 * RS + j];
        step(rb);
      }
      if (left) step(ra);
    }
  } else {
    // runs of the cubic phase recurrence (see PhaseRuns).  A walk that
    // starts inside a run (a chunk, or a wave's share of one) first advances
    // the run's table down to its own first bin without accumulating.
    const double lin_step = -c.a8 * df;  // linear phase change per bin of the descending walk
    constexpr int US = 2 * ND;
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
      if (L == 0) {
        // below the lowest level: every bin evaluated directly
        const int nd = k - kb + 1 < 4 ? k - kb + 1 : 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (j < nd) {
            const double* __restrict__ rc = bins + (int64_t)(k - j) * RS;
            const double r = phase_nonlinear(c, rc[0], rc[1], rc[2], rc[3]) + fma(c.a8, rc[0] * rc[1], c.a5);
            double gr, gi;
            phasor<PREC>(r, T, &gr, &gi);
            accumulate(rc + 4, gr, gi);
          }
        }
        k -= nd;
        continue;
      }
      const int top = s + L - 1 < n_freq - 1 ? s + L - 1 : n_freq - 1;
      const int nd = top - s + 1 < 4 ? top - s + 1 : 4;
      // the run's first (up to) four bins, evaluated directly; their
      // nonlinear parts build the backward differences n0..n3
      double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0, lin = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j < nd) {
          const int kk = top - j;
          const double* __restrict__ rc = bins + (int64_t)kk * RS;
          const double nl = phase_nonlinear(c, rc[0], rc[1], rc[2], rc[3]);
          lin = fma(c.a8, rc[0] * rc[1], c.a5);
          const double d1 = nl - n0;
          const double d2 = d1 - n1;
          n3 = d2 - n2;
          n2 = d2;
          n1 = d1;
          n0 = nl;
          if (kk <= k && kk >= kb) {
            double gr, gi;
            phasor<PREC>(nl + lin, T, &gr, &gi);
            accumulate(rc + 4, gr, gi);
          }
        }
      }
      const int lo = s > kb ? s : kb;  // the run's last bin in this walk
      int kk = top - nd;
      if (kk >= lo) {
        // the remaining bins from the table of the full phase
        double p0 = n0 + lin, p1 = n1 + lin_step, p2 = n2;
        const double p3 = n3;
        for (; kk > k; --kk) {  // above the walk's first bin: advance only
          p2 += p3;
          p1 += p2;
          p0 += p1;
        }
        auto step = [&](const double* __restrict__ u) {
          p2 += p3;
          p1 += p2;
          p0 += p1;
          double gr, gi;
          phasor<PREC>(p0, T, &gr, &gi);
          accumulate(u, gr, gi);
        };
        // bins in pairs, one loop exit, so that the accumulators of the
        // two steps can alternate registers; the next record is in flight
        // while one is processed
        double ua[US], ub[US];
#pragma unroll
        for (int j = 0; j < US; ++j) ua[j] = bins[(int64_t)kk * RS + 4 + j];
        int left = kk - lo + 1;
        for (; left >= 2; left -= 2, kk -= 2) {
#pragma unroll
          for (int j = 0; j < US; ++j) ub[j] = bins[(int64_t)(kk - 1) * RS + 4 + j];
          step(ua);
          const int k2 = kk - 2 >= lo ? kk - 2 : lo;
#pragma unroll
          for (int j = 0; j < US; ++j) ua[j] = bins[(int64_t)k2 * RS + 4 + j];
          step(ub);
        }
        if (left) step(ua);
      }
      k = s - 1;
    }
  }
  // Apply exp(-2 pi i f_kb (tau_i - tau_0)) to the recurrences.
#pragma unroll
  for (int i = 1; i < ND; ++i) {
    const double dt = coef[(C_DT1 + i - 1) * ld + pc];
    const double fb = (double)(k0 + kb) * df;
    double s, co;
    sincos_cycles(fb * dt, T, &s, &co);
    const double er = co, ei = -s;
    const double tr = zr[i] * er - zi[i] * ei;
    const double ti = zr[i] * ei + zi[i] * er;
    zr[i] = tr;
    zi[i] = ti;
  }
  if (PREC == 1) {
    // remove the mean bias of the hardware phasor (every sum is linear in it)
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const double tr = zr[i] * pg_re - zi[i] * pg_im;
      zi[i] = zr[i] * pg_im + zi[i] * pg_re;
      zr[i] = tr;
    }
  }
  if constexpr (LIST) {
    if (!wave_sums_combine<ND>(zr, zi)) return;
  }
  if (live) {
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      partial[((int64_t)chunk * 2 * ND + 2 * i) * n + p] = zr[i];
      partial[((int64_t)chunk * 2 * ND + 2 * i + 1) * n + p] = zi[i];
    }
  }
}

constexpr int kWMom = 12;          // Chebyshev orders per block and detector
static_assert(kWMom % 2 == 0, "the few-slot build reads the orders in pairs");
constexpr int64_t kWBuildManyRows = 512;  // builds listing fewer slots use k_wmom_build_few
constexpr double kTauCap = 0.25;    // largest |t_c + dt_i| (s) the moment cache is built for

// Extrinsic moves with a cached waveform (Sec. III.B: the fast blocks reuse
// the waveform of the chain's intrinsic parameters and only redo the
// projection).  A fast row changes only the detector delays
// tau_i = t_c + dt_i (and the per-detector factors A P_i applied later), so
//   z_i = sum_k u_ik g_k exp(-2 pi i f_k tau_i),
// g_k = exp(-2 pi i Psi(f_k)) the slot's intrinsic phasor (Psi without the
// linear time term).  Over a block of B bins with centre f_c and
// t_j = (j - (B - 1) / 2) / (B / 2) in [-1, 1],
//   exp(-2 pi i f_k tau) = E exp(-i phi t_j),  E = exp(-2 pi i f_c tau),
//   phi = pi df B tau,
// and exp(-i phi t) = sum_m eps_m (-i)^m J_m(phi) T_m(t) (Jacobi-Anger,
// eps_0 = 1, eps_m = 2), so each block contributes
// E sum_m eps_m (-i)^m J_m(phi) M_m with the slot's Chebyshev moments
// M_m = sum_j T_m(t_j) u_ij g_j (m < kWMom).  The moments depend on the slot
// only: they are built once per slot (k_wmom_build, FP64 sums rounded to FP32)
// and a fast row costs kWMom terms per block and detector instead of B bins.
// B is chosen so that |phi| <= 1.61 for |tau| <= kTauCap, where the dropped
// orders stay below 2 (phi / 2)^12 / 12! = 3e-10 of the block's sum of |u g|
// (the FP32 moments carry 6e-8); rows with a larger |tau_i| are flagged (NaN).
//
// Slot layout: float2 [n_blk][n_det][kWMom].

// t[m] = eps_m J_m(x) with the sign of (-i)^m folded in (+ for m mod 4 in
// {0, 1}, - otherwise), m < kWMom, |x| <= 1.61: the power series of J_m, 14
// terms (the last below 3e-14 of the first).
__device__ inline void wmom_coefs(double x, double* t) {
  const double h = 0.5 * x, y = -h * h;
  double lead = 1.0;  // (x / 2)^m / m!
#pragma unroll
  for (int m = 0; m < kWMom; ++m) {
    double term = 1.0, sum = 1.0;
#pragma unroll
    for (int k = 1; k <= 14; ++k) {
      term *= y * (1.0 / (double)(k * (m + k)));
      sum += term;
    }
    const double j = lead * sum * (m == 0 ? 1.0 : 2.0);
    t[m] = (m & 3) < 2 ? j : -j;
    lead *= h * (1.0 / (double)(m + 1));
  }
}

// k_wmom_build: lane = listed slot (64 per workgroup), workgroup = (block,
// slot tile); the block's bins are walked from the top (wave-uniform
// records) as in the time-marginal moments: FP64 phase and sin/cos for
// PREC = 0, the mixed form's phase recurrence in runs and the FP32 hardware
// sin/cos for PREC = 1 (the moments are stored in FP32 either way); FP64
// sums.  Tiles at or beyond the device-side count exit at once.
template <int ND, int PREC>
__global__ void __launch_bounds__(64) k_wmom_build(const double* __restrict__ coef, int64_t ld,
                                                   const int32_t* __restrict__ slots,
                                                   const int32_t* __restrict__ count, int rows_per_slot,
                                                   const int32_t* __restrict__ src, const double* __restrict__ bins,
                                                   int n_freq, int blk, int64_t slot_f2, TrigConsts T, PhaseRuns R,
                                                   double pg_re, double pg_im, const double* __restrict__ basis,
                                                   float2* __restrict__ mom) {
  constexpr int RS = 4 + 2 * ND;
  const int b = blockIdx.x, tile = blockIdx.y;
  const int cnt = *count;
  if (tile * 64 >= cnt) return;  // uniform over the workgroup
  const int li = tile * 64 + (int)threadIdx.x;
  const int sl = li < cnt ? slots[li] : -1;
  int64_t r = 0;  // coefficient row; row 0 for lanes that store nothing
  if (sl >= 0) r = src ? (int64_t)src[li] : (int64_t)sl * rows_per_slot;
  PhaseCoef c;
  c.a0 = coef[C_A0 * ld + r];
  c.a2 = coef[C_A2 * ld + r];
  c.a3 = coef[C_A3 * ld + r];
  c.a4 = coef[C_A4 * ld + r];
  c.a5 = coef[C_A5 * ld + r];
  c.a6 = coef[C_A6 * ld + r];
  c.a7 = coef[C_A7 * ld + r];
  c.a8 = 0.0;  // the linear time term is applied per row
  c.a10 = coef[C_A10 * ld + r];
  c.a12 = coef[C_A12 * ld + r];
  c.b5 = coef[C_B5 * ld + r];
  c.b6 = coef[C_B6 * ld + r];
  const int kb = b * blk;
  const int ke = kb + blk < n_freq ? kb + blk : n_freq;
  double mr[ND][kWMom], mi[ND][kWMom];
#pragma unroll
  for (int i = 0; i < ND; ++i)
#pragma unroll
    for (int m = 0; m < kWMom; ++m) mr[i][m] = mi[i][m] = 0.0;
  auto visit = [&](int k, double gr, double gi) {
    const double* __restrict__ u = bins + (int64_t)k * RS + 4;
    const double* __restrict__ tq = basis + (int64_t)(k - kb) * kWMom;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const double ur = u[2 * i], ui = u[2 * i + 1];
      const double wr = ur * gr - ui * gi, wi = ur * gi + ui * gr;
#pragma unroll
      for (int m = 0; m < kWMom; ++m) {
        mr[i][m] = fma(tq[m], wr, mr[i][m]);
        mi[i][m] = fma(tq[m], wi, mi[i][m]);
      }
    }
  };
  if constexpr (PREC == 0) {
    for (int k = ke - 1; k >= kb; --k) {
      const double* __restrict__ rc = bins + (int64_t)k * RS;
      double sn, cs;
      sincos_cycles(phase_cycles(c, rc[0], rc[1], rc[2], rc[3]), T, &sn, &cs);
      visit(k, cs, -sn);
    }
  } else {
    // the runs of the mixed walk, as in k_tmom: one visit site per bin
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
      const int top = L == 0 ? k : (s + L - 1 < n_freq - 1 ? s + L - 1 : n_freq - 1);
      if (L == 0) s = k;
      const int nd = top - s + 1 < 4 ? top - s + 1 : 4;
      double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
      double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0;
#pragma nounroll
      for (int j = 0; j < nd; ++j) {
        const double* __restrict__ rc = bins + (int64_t)(top - j) * RS;
        const double nl = phase_nonlinear(c, rc[0], rc[1], rc[2], rc[3]);
        const double d1 = nl - n0;
        const double d2 = d1 - n1;
        n3 = d2 - n2;
        n2 = d2;
        n1 = d1;
        n0 = nl;
        const double ph = nl + c.a5;
        r0 = j == 0 ? ph : r0;
        r1 = j == 1 ? ph : r1;
        r2 = j == 2 ? ph : r2;
        r3 = j == 3 ? ph : r3;
      }
      double p0 = n0 + c.a5, p1 = n1, p2 = n2;
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
        const float t = (float)(ph - rint(ph));
        visit(kk, (double)__builtin_amdgcn_cosf(t), -(double)__builtin_amdgcn_sinf(t));
      }
      k = s - 1;
    }
  }
  if (sl < 0) return;
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    float2* __restrict__ out = mom + sl * slot_f2 + ((int64_t)b * ND + i) * kWMom;
#pragma unroll
    for (int m = 0; m < kWMom; ++m) {
      double vr = mr[i][m], vi = mi[i][m];
      if (PREC == 1) {  // remove the mean bias of the hardware phasor
        const double tr = vr * pg_re - vi * pg_im;
        vi = vr * pg_im + vi * pg_re;
        vr = tr;
      }
      out[m] = make_float2((float)vr, (float)vi);
    }
  }
}

// k_wmom_build_few: the same moments for the sampler's rounds, where a few
// listed slots rebuild at a time; the work follows the device-side count.  A
// unit is (block, group of kWBuildSlots listed slots), units ordered so that
// neighbouring workgroups share a block (its records stay in L2); the grid
// strides over the units.  Per unit: the group's phase coefficients go to
// LDS (one load per thread), then thread k evaluates bin k's phasor for every
// slot of the group (FP64 phase; FP64 or FP32 hardware sin/cos) and stages
// the bin's projected data, all in LDS; lane (slot, detector, part) then sums
// the moments over bins part, part + Q, ... (Q = min(16, blk) parts, FP64),
// so that the 16 lanes of a (slot, detector) read 16 consecutive bins of each
// LDS array (no bank conflicts), and the Q partial sums are added by lane
// exchange in a fixed order.  The Chebyshev values are copied to LDS once per
// workgroup, as pairs (T_2j, T_2j+1) per bin.  Dynamic LDS:
// blk (16 kWBuildSlots + 16 nd + 8 kWMom) bytes + the coefficients.
constexpr int kWBuildSlots = 4;
constexpr int kWBuildCoef = 12;  // phase coefficients per slot

inline size_t wmom_build_few_lds(int blk, int nd) {
  return (size_t)blk * (16 * kWBuildSlots + 16 * nd + 8 * kWMom) + 8 * kWBuildSlots * kWBuildCoef;
}

template <int PREC>
__global__ void __launch_bounds__(256) k_wmom_build_few(const double* __restrict__ coef, int64_t ld,
                                                        const int32_t* __restrict__ slots,
                                                        const int32_t* __restrict__ count, int rows_per_slot,
                                                        const int32_t* __restrict__ src,
                                                        const double* __restrict__ bins, int rs, int n_freq, int nd,
                                                        int blk, int n_blk, int64_t slot_f2, TrigConsts T,
                                                        double pg_re, double pg_im,
                                                        const double* __restrict__ basis, float2* __restrict__ mom) {
  extern __shared__ __attribute__((aligned(16))) double lds[];
  double2* g_lds = reinterpret_cast<double2*>(lds);   // [kWBuildSlots][blk]
  double* u_lds = lds + 2 * kWBuildSlots * blk;        // [blk][2 nd]
  double2* t_lds = reinterpret_cast<double2*>(u_lds + 2 * nd * blk);  // [kWMom / 2][blk]
  double* c_lds = u_lds + 2 * nd * blk + kWMom * blk;  // [kWBuildSlots][kWBuildCoef]
  const int cnt = *count;
  const int ngrp = (cnt + kWBuildSlots - 1) / kWBuildSlots;
  const int64_t units = (int64_t)n_blk * ngrp;
  if (units <= blockIdx.x) return;
  const int Q = blk < 16 ? blk : 16;  // power of two: parts per (slot, detector)
  const int tid = threadIdx.x;
  const int part = tid % Q, combo = tid / Q;
  const int s_me = combo / nd, i_me = combo - (combo / nd) * nd;
  const bool lane_on = s_me < kWBuildSlots;  // Q kWBuildSlots nd <= 256 for nd <= 4
  constexpr int kCoefIdx[kWBuildCoef] = {C_A0, C_A2, C_A3, C_A4, C_A5, C_A6, C_A7, C_A10, C_A12, C_B5, C_B6, C_A0};
  for (int e = tid; e < blk * (kWMom / 2); e += blockDim.x) {
    const int j = e / blk, k = e - j * blk;
    t_lds[e] = make_double2(basis[k * kWMom + 2 * j], basis[k * kWMom + 2 * j + 1]);
  }
  for (int64_t unit = blockIdx.x; unit < units; unit += gridDim.x) {
    const int b = (int)(unit / ngrp), grp = (int)(unit - (int64_t)b * ngrp);
    const int kb = b * blk;
    const int nbin = kb + blk < n_freq ? blk : n_freq - kb;
    __syncthreads();  // the previous unit's LDS contents are consumed
    if (tid < kWBuildSlots * kWBuildCoef) {
      const int s = tid / kWBuildCoef, j = tid - s * kWBuildCoef;
      const int li = grp * kWBuildSlots + s;
      double v = 0.0;
      if (li < cnt && slots[li] >= 0 && j < 11) {
        const int64_t r = src ? (int64_t)src[li] : (int64_t)slots[li] * rows_per_slot;
        v = coef[kCoefIdx[j] * ld + r];
      }
      c_lds[tid] = v;
    }
    __syncthreads();
    for (int k = tid; k < blk; k += blockDim.x) {
      const double* rec = bins + (int64_t)(kb + (k < nbin ? k : 0)) * rs;
      const double x = rec[0], x2 = rec[1], xm5 = rec[2], lnf = rec[3];
      for (int j = 0; j < 2 * nd; ++j) u_lds[k * 2 * nd + j] = k < nbin ? rec[4 + j] : 0.0;
#pragma unroll
      for (int s = 0; s < kWBuildSlots; ++s) {
        const int li = grp * kWBuildSlots + s;
        double2 g = make_double2(0.0, 0.0);
        if (li < cnt && k < nbin && slots[li] >= 0) {
          const double* cs = c_lds + s * kWBuildCoef;
          PhaseCoef c;
          c.a0 = cs[0];
          c.a2 = cs[1];
          c.a3 = cs[2];
          c.a4 = cs[3];
          c.a5 = cs[4];
          c.a6 = cs[5];
          c.a7 = cs[6];
          c.a8 = 0.0;  // the linear time term is applied per row
          c.a10 = cs[7];
          c.a12 = cs[8];
          c.b5 = cs[9];
          c.b6 = cs[10];
          const double ph = phase_cycles(c, x, x2, xm5, lnf);
          if (PREC == 0) {
            double sn, csn;
            sincos_cycles(ph, T, &sn, &csn);
            g = make_double2(csn, -sn);
          } else {
            const float t = (float)(ph - rint(ph));
            g = make_double2((double)__builtin_amdgcn_cosf(t), -(double)__builtin_amdgcn_sinf(t));
          }
        }
        g_lds[s * blk + k] = g;
      }
    }
    __syncthreads();
    const int li = grp * kWBuildSlots + s_me;
    const int64_t sl = lane_on && li < cnt ? slots[li] : -1;
    double mr[kWMom], mi[kWMom];
#pragma unroll
    for (int m = 0; m < kWMom; ++m) mr[m] = mi[m] = 0.0;
    if (sl >= 0) {
      for (int k = part; k < nbin; k += Q) {
        const double2 g = g_lds[s_me * blk + k];
        const double2 u = *reinterpret_cast<const double2*>(u_lds + k * 2 * nd + 2 * i_me);
        const double wr = u.x * g.x - u.y * g.y, wi = u.x * g.y + u.y * g.x;
#pragma unroll
        for (int j = 0; j < kWMom / 2; ++j) {
          const double2 t = t_lds[j * blk + k];
          mr[2 * j] = fma(t.x, wr, mr[2 * j]);
          mi[2 * j] = fma(t.x, wi, mi[2 * j]);
          mr[2 * j + 1] = fma(t.y, wr, mr[2 * j + 1]);
          mi[2 * j + 1] = fma(t.y, wi, mi[2 * j + 1]);
        }
      }
    }
    // parts sit in consecutive lanes: pairwise sums in a fixed order
    for (int off = 1; off < Q; off <<= 1) {
#pragma unroll
      for (int m = 0; m < kWMom; ++m) {
        mr[m] += __shfl_xor(mr[m], off);
        mi[m] += __shfl_xor(mi[m], off);
      }
    }
    if (sl >= 0 && part == 0) {
      float2* __restrict__ out = mom + sl * slot_f2 + ((int64_t)b * nd + i_me) * kWMom;
#pragma unroll
      for (int m = 0; m < kWMom; ++m) {
        double vr = mr[m], vi = mi[m];
        if (PREC == 1) {  // remove the mean bias of the hardware phasor
          const double tr = vr * pg_re - vi * pg_im;
          vi = vr * pg_im + vi * pg_re;
          vr = tr;
        }
        out[m] = make_float2((float)vr, (float)vi);
      }
    }
  }
}

// k_wmom: the fast reduction.  Lane = row (rows[0 .. *count), 64 to a
// workgroup, slot slot_of[p] or p / rows_per_slot); the workgroup owns a chunk
// of blocks that its waves split, their sums added in wave order; chunk
// partials as k_full's ([chunk][2 ND][n]).  Each lane streams its slot's
// moments, 96 bytes per detector and block.  With n_out > n_chunks the
// partials fill the first n_chunks of a layout of n_out chunks (that of the
// full reduction of the same round) and the rest are written zero, so the
// common epilogue sums them.
template <int ND>
__global__ void __launch_bounds__(256) k_wmom(const double* __restrict__ coef, int64_t ld, int64_t n, int64_t k0,
                                              double df, int blk, int n_blk, int n_chunks, int n_out, TrigConsts T,
                                              const int32_t* __restrict__ rows, const int32_t* __restrict__ count,
                                              int rows_per_slot, const int32_t* __restrict__ slot_of,
                                              const float2* __restrict__ mom, int64_t slot_f2,
                                              double* __restrict__ partial) {
  const int nptile = (int)((n + 63) / 64);
  int chunk, ptile;
  decode_block(blockIdx.x, nptile, n_chunks, &chunk, &ptile);
  const int cnt = *count;
  if (ptile * 64 >= cnt) return;  // uniform over the workgroup
  const int idx = ptile * 64 + (threadIdx.x & 63);
  const bool live = idx < cnt;
  const int64_t p = rows[live ? idx : cnt - 1];
  int64_t slot = slot_of ? (int64_t)slot_of[p] : p / rows_per_slot;
  if (slot < 0) slot = 0;  // a row without a valid slot (the caller discards it)
  const float4* __restrict__ ms = reinterpret_cast<const float4*>(mom + slot * slot_f2);

  // this wave's blocks
  const int per = (n_blk + n_chunks - 1) / n_chunks;
  const int nw = blockDim.x >> 6, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cb = chunk * per, ce = cb + per < n_blk ? cb + per : n_blk;
  const int sub = ((ce > cb ? ce - cb : 0) + nw - 1) / nw;
  const int bb = cb + wv * sub, be = bb + sub < ce ? bb + sub : ce;

  const double tau0 = coef[C_TAU0 * ld + p];
  double zr[ND], zi[ND], er[ND], ei[ND], rr[ND], ri[ND], tc[ND][kWMom];
  bool in_range = true;
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    const double tau = i == 0 ? tau0 : tau0 + coef[(C_DT1 + i - 1) * ld + p];
    in_range = in_range && fabs(tau) <= kTauCap;
    wmom_coefs(kPi * df * blk * (fabs(tau) <= kTauCap ? tau : 0.0), tc[i]);
    double sn, cs;
    // E at the centre of the first block, and the block-to-block rotation
    sincos_cycles(((double)k0 + (double)bb * blk + 0.5 * (blk - 1)) * df * tau, T, &sn, &cs);
    er[i] = cs;
    ei[i] = -sn;
    sincos_cycles((double)blk * df * tau, T, &sn, &cs);
    rr[i] = cs;
    ri[i] = -sn;
    zr[i] = 0.0;
    zi[i] = 0.0;
  }
  for (int b = bb; b < be; ++b) {
    const float4* __restrict__ mb = ms + (int64_t)b * ND * (kWMom / 2);
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      float4 v[kWMom / 2];
#pragma unroll
      for (int q = 0; q < kWMom / 2; ++q) v[q] = mb[i * (kWMom / 2) + q];
      // H = sum_m eps_m (-i)^m J_m(phi) M_m (signs folded into tc)
      double hr = 0.0, hi = 0.0;
#pragma unroll
      for (int m = 0; m < kWMom; ++m) {
        const double mre = (double)((m & 1) ? v[m >> 1].z : v[m >> 1].x);
        const double mim = (double)((m & 1) ? v[m >> 1].w : v[m >> 1].y);
        if ((m & 1) == 0) {
          hr = fma(tc[i][m], mre, hr);
          hi = fma(tc[i][m], mim, hi);
        } else {
          hr = fma(tc[i][m], mim, hr);
          hi = fma(-tc[i][m], mre, hi);
        }
      }
      zr[i] = fma(er[i], hr, zr[i]);
      zr[i] = fma(-ei[i], hi, zr[i]);
      zi[i] = fma(er[i], hi, zi[i]);
      zi[i] = fma(ei[i], hr, zi[i]);
      const double tr = er[i] * rr[i] - ei[i] * ri[i];
      ei[i] = er[i] * ri[i] + ei[i] * rr[i];
      er[i] = tr;
    }
  }
  if (!in_range) {
#pragma unroll
    for (int i = 0; i < ND; ++i) zr[i] = zi[i] = __builtin_nan("");
  }
  if (!wave_sums_combine<ND>(zr, zi)) return;
  if (live) {
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      partial[((int64_t)chunk * 2 * ND + 2 * i) * n + p] = zr[i];
      partial[((int64_t)chunk * 2 * ND + 2 * i + 1) * n + p] = zi[i];
    }
    for (int c = n_chunks + chunk; c < n_out; c += n_chunks)
#pragma unroll
      for (int j = 0; j < 2 * ND; ++j) partial[((int64_t)c * 2 * ND + j) * n + p] = 0.0;
  }
}

// Sum the fast rows' chunk partials (fixed order) into zout[p][2 nd]: one
// lane per (listed row, component).
__global__ void __launch_bounds__(256) k_wmom_sum(const double* __restrict__ partial, int n_chunks, int nd, int64_t n,
                                                  const int32_t* __restrict__ rows,
                                                  const int32_t* __restrict__ count, double* __restrict__ zout) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int idx = t / (2 * nd), j = t - idx * (2 * nd);
  if (idx >= *count) return;
  const int64_t p = rows[idx];
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  int c = 0;
  for (; c + 8 <= n_chunks; c += 8) {
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] += partial[((int64_t)(c + q) * 2 * nd + j) * n + p];
  }
  for (int q = 0; c + q < n_chunks; ++q) acc[q] += partial[((int64_t)(c + q) * 2 * nd + j) * n + p];
  zout[p * 2 * nd + j] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// Matrix-core form of the mixed reduction.
//
// Within a block of B bins (k = b0 + j) with centre c = (B - 1) / 2 the delay
// rotation of detector i is expanded in t_j = (j - c) / (B / 2):
//   e^{-2 pi i f_k tau_i} = E_ib sum_m (-i phi_i)^m t_j^m / m!,
//   E_ib = e^{-2 pi i f_centre tau_i},  phi_i = pi df tau_i B,
// and B is chosen so that |phi_i| keeps the first dropped term below 1e-9.
// The block sums then become moments M_iq = sum_j W_q[k] g_k of the phasors
// g_k = e^{-2 pi i Phi_0(f_k)} with proposal-independent weights
// W_q[k] = t_j^m u_ik: a dense [proposals x bins] x [bins x 16] contraction per
// block, done by v_mfma_f32_16x16x4_f32 in the three-multiplication complex
// form (k1 = (g_r + g_i) w_r, k2 = g_r (w_i - w_r), k3 = g_i (w_r + w_i);
// re = k1 - k3, im = k1 + k2).  Lane l of a wave computes the phasor of
// proposal (l mod 16) of each of its MT 16-row tiles at bin (l / 16) of each
// 4-bin step, which is exactly the MFMA A-operand layout.  After each block the
// 16 x 16 FP32 accumulators go through LDS to one lane per proposal, which
// folds them into FP64 sums with the block factor E_ib (phase reduced in FP64,
// FP32 hardware sin/cos as for the phasors).  Partials have the layout of
// k_full.
constexpr int kMomCols = 16;

template <int ND>
struct MomCount {
  static constexpr int value = ND > 1 ? (kMomCols - 1) / (ND - 1) : 0;
};

// 4 x 4 transpose between the 16-lane rows of a wave and four registers:
// afterwards v[j] in row R holds what v[R] held in row j (same column).
__device__ inline void transpose_rows4(float v[4]) {
  auto sw32 = [](float& a, float& b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
  };
  auto sw16 = [](float& a, float& b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
  };
  sw32(v[0], v[2]);
  sw32(v[1], v[3]);
  sw16(v[0], v[1]);
  sw16(v[2], v[3]);
}

// Lane l owns proposal l of its wave for the whole walk, as in k_full; the
// bin records of a 4-bin step are wave-uniform (scalar loads).  Each lane
// computes its proposal's phasor at the 4 bins (four independent FP64 phase
// evaluations); a row/register transpose then gives, for each 16-proposal
// tile mt, the A operand of v_mfma_f32_16x16x4_f32 (lane r + 16 R: proposal
// 16 mt + r at bin R), and the B operand is the weight row of bin (lane / 16),
// column (lane mod 16).
template <int ND>
__global__ void __launch_bounds__(256) k_full_mfma(const double* __restrict__ coef, int64_t ld, int64_t n,
                                                   const double* __restrict__ bins, const float* __restrict__ wtab,
                                                   int64_t k0, double df, int n_freq, int n_pad, int blk,
                                                   int chunk_len, int n_chunks, double pg_re, double pg_im,
                                                   double* __restrict__ partial) {
  constexpr int RS = 4 + 2 * ND;
  constexpr int KM = MomCount<ND>::value;
  constexpr int RW = 3 * kMomCols + 1;  // LDS row stride (floats), odd against bank conflicts
  __shared__ float red[4][64][RW];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int tpb = blockDim.x;
  const int nptile = (int)((n + tpb - 1) / tpb);
  int chunk, ptile;
  decode_block(blockIdx.x, nptile, n_chunks, &chunk, &ptile);
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

  const int kb = chunk * chunk_len;
  const int ke = kb + chunk_len < n_pad ? kb + chunk_len : n_pad;
  double zr[ND], zi[ND], tau[ND];
  float phi[ND];
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    zr[i] = 0.0;
    zi[i] = 0.0;
    tau[i] = 0.0;
    phi[i] = 0.0f;
  }
#pragma unroll
  for (int i = 1; i < ND; ++i) {
    tau[i] = coef[(C_DT1 + i - 1) * ld + pc];
    phi[i] = (float)(kPi * df * tau[i] * (double)blk);
  }
  typedef float f4v __attribute__((ext_vector_type(4)));
  f4v acc[4][3];
  auto load_w = [&](int k, float* w) {
    k = k < n_pad ? k : n_pad - 1;
    const float* src = wtab + ((int64_t)k * kMomCols + (lane & 15)) * 3;
    w[0] = src[0];
    w[1] = src[1];
    w[2] = src[2];
  };
  // Phase records of the 4 bins of a step (wave-uniform, scalar loads).
  struct Recs {
    double v[4][4];
  };
  auto load_recs = [&](int kq, Recs& r) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int k = kq + b < n_freq ? kq + b : n_freq - 1;
      const double* rec = bins + (int64_t)k * RS;
#pragma unroll
      for (int j = 0; j < 4; ++j) r.v[b][j] = rec[j];
    }
  };
  float wa[3], wb[3];
  Recs ra, rb;
  load_w(kb + (lane >> 4), wa);
  load_recs(kb, ra);
  // One 4-bin step with records r and weights w (this lane's column).
  auto step = [&](const Recs& rc, const float* w) {
    float gr[4], gi[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double r = phase_cycles(c, rc.v[b][0], rc.v[b][1], rc.v[b][2], rc.v[b][3]);
      const float tf = (float)(r - rint(r));
      gr[b] = __builtin_amdgcn_cosf(tf);
      gi[b] = -__builtin_amdgcn_sinf(tf);
    }
    transpose_rows4(gr);
    transpose_rows4(gi);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      acc[mt][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(gr[mt] + gi[mt], w[0], acc[mt][0], 0, 0, 0);
      acc[mt][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(gr[mt], w[1], acc[mt][1], 0, 0, 0);
      acc[mt][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(gi[mt], w[2], acc[mt][2], 0, 0, 0);
    }
  };
  for (int b0 = kb; b0 < ke; b0 += blk) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int t = 0; t < 3; ++t) acc[mt][t] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
    // blk is a multiple of 8: steps pair up, each one's operands loaded
    // while the other computes.  Scalar loads complete out of order, so the
    // only usable wait is lgkmcnt(0): it is placed before the other set's loads
    // are issued, so that it never waits for a load issued just before it.
    // The last loads run ahead into the next block.
    for (int s = 0; s < blk; s += 8) {
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): set a is in
      load_w(b0 + s + 4 + (lane >> 4), wb);
      load_recs(b0 + s + 4, rb);
      __builtin_amdgcn_sched_barrier(0);
      step(ra, wa);
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_waitcnt(0xC07F);  // set b is in
      load_w(b0 + s + 8 + (lane >> 4), wa);
      load_recs(b0 + s + 8, ra);
      __builtin_amdgcn_sched_barrier(0);
      step(rb, wb);
      __builtin_amdgcn_sched_barrier(0);
    }
    // D[row = 4 (lane / 16) + v][column = lane mod 16] of tile mt is proposal
    // 16 mt + row, moment column q.
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          red[wave][mt * 16 + 4 * (lane >> 4) + v][t * kMomCols + (lane & 15)] = acc[mt][t][v];
    __syncthreads();
    {
      const float* rw = red[wave][lane];
      // detector 0: column 0, no rotation
      zr[0] += (double)(rw[0] - rw[2 * kMomCols]);
      zi[0] += (double)(rw[0] + rw[kMomCols]);
#pragma unroll
      for (int i = 1; i < ND; ++i) {
        // S_i = sum_m (-i phi)^m / m! * M_i,m by a Horner sweep from the top moment
        float sr = 0.0f, si = 0.0f;
#pragma unroll
        for (int m = KM - 1; m >= 0; --m) {
          const int q = 1 + (i - 1) * KM + m;
          const float mr = rw[q] - rw[2 * kMomCols + q];
          const float mi = rw[q] + rw[kMomCols + q];
          const float f = phi[i] / (float)(m + 1);  // s <- s (-i phi / (m + 1)) + M_m
          const float nr = si * f + mr;
          const float ni = -sr * f + mi;
          sr = nr;
          si = ni;
        }
        // block factor E = exp(-2 pi i f_centre tau_i): FP64 reduction to a
        // fraction of a cycle, FP32 hardware sin/cos
        const double cyc = ((double)(k0 + b0) + 0.5 * (double)(blk - 1)) * df * tau[i];
        const float tf = (float)(cyc - rint(cyc));
        const double er = (double)__builtin_amdgcn_cosf(tf), ei = -(double)__builtin_amdgcn_sinf(tf);
        const double dr = (double)sr, di = (double)si;
        zr[i] = fma(er, dr, fma(-ei, di, zr[i]));
        zi[i] = fma(er, di, fma(ei, dr, zi[i]));
      }
    }
    __syncthreads();
  }
  // remove the mean bias of the hardware phasor: once in the phasors, once
  // more in the block factors of detectors 1..
  {
    const double g2r = pg_re * pg_re - pg_im * pg_im, g2i = 2.0 * pg_re * pg_im;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const double gr = i == 0 ? pg_re : g2r, gi = i == 0 ? pg_im : g2i;
      const double tr = zr[i] * gr - zi[i] * gi;
      zi[i] = zr[i] * gi + zi[i] * gr;
      zr[i] = tr;
    }
  }
  if (p < n) {
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      partial[((int64_t)chunk * 2 * ND + 2 * i) * n + p] = zr[i];
      partial[((int64_t)chunk * 2 * ND + 2 * i + 1) * n + p] = zi[i];
    }
  }
}

// Combine the chunk partials and apply the marginalisation.  A workgroup
// takes 64 proposals; its 16 waves sum the chunks c = w (mod 16) in order and
// wave 0 adds the sixteen sums in order, so the result is reproducible.  For the
// distance marginal this writes (|Z_1|, <h|h>_1) for k_dist_marg.  With a
// waveform cache, a row p with zsrc[p] >= 0 takes its sums z_i from slot
// zsrc[p] of zc ([slot][2 nd]) instead of the partials (moves that change only
// A P_i), and zrow (when not NULL) receives every row's z_i ([n][2 nd]).
// The partials of chunk c are read at chunk index c * cstride (1, or the
// group length after k_partial_reduce).
__global__ void __launch_bounds__(1024) k_epilogue(const double* __restrict__ partial, int n_chunks, int cstride,
                                                  int nd, const double* __restrict__ coef, int64_t ld, int64_t n,
                                                  double dd, int marg, double* __restrict__ logl,
                                                  double* __restrict__ zbuf, const int32_t* __restrict__ zsrc,
                                                  const double* __restrict__ zc, double* __restrict__ zrow) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * 64 + lane;
  const int64_t pc = p < n ? p : n - 1;
  double z[2 * kMaxDet];
#pragma unroll
  for (int j = 0; j < 2 * kMaxDet; ++j) z[j] = 0.0;
  for (int c = wave; c < n_chunks; c += 16) {
#pragma unroll
    for (int j = 0; j < 2 * kMaxDet; ++j)
      if (j < 2 * nd) z[j] += partial[((int64_t)c * cstride * 2 * nd + j) * n + pc];
  }
  __shared__ double red[15][2 * kMaxDet][64];
  if (wave > 0) {
#pragma unroll
    for (int j = 0; j < 2 * kMaxDet; ++j) red[wave - 1][j][lane] = z[j];
  }
  __syncthreads();
  if (wave != 0 || p >= n) return;
  for (int w = 0; w < 15; ++w)
#pragma unroll
    for (int j = 0; j < 2 * kMaxDet; ++j) z[j] += red[w][j][lane];
  if (zsrc) {
    const int32_t sl = zsrc[p];
    if (sl >= 0) {
#pragma unroll
      for (int j = 0; j < 2 * kMaxDet; ++j)
        if (j < 2 * nd) z[j] = zc[(int64_t)sl * 2 * nd + j];
    }
  }
  if (zrow) {
#pragma unroll
    for (int j = 0; j < 2 * kMaxDet; ++j)
      if (j < 2 * nd) zrow[p * 2 * nd + j] = z[j];
  }
  const bool valid = coef[C_VALID * ld + p] != 0.0;
  double Zr = 0.0, Zi = 0.0, plain = 0.0;
#pragma unroll
  for (int i = 0; i < kMaxDet; ++i) {
    if (i >= nd) break;
    const double zr = z[2 * i], zi = z[2 * i + 1];
    const double ar = coef[(C_APRE + i) * ld + p];
    const double ai = coef[(C_APIM + i) * ld + p];
    const double hr = ar * zr - ai * zi;
    const double hi = ar * zi + ai * zr;
    plain += hr;
    Zr += hr;
    Zi += hi;
  }
  const double hh = coef[C_HH * ld + p];
  if (marg == 2) {
    zbuf[p] = valid ? sqrt(Zr * Zr + Zi * Zi) : -1.0;
    zbuf[n + p] = hh;
    return;
  }
  double out;
  if (!valid) {
    out = -INFINITY;
  } else if (marg == 0) {
    out = -0.5 * dd + plain - 0.5 * hh;
  } else {
    out = -0.5 * dd - 0.5 * hh + log_i0(sqrt(Zr * Zr + Zi * Zi));
  }
  logl[p] = out;
}

// First level of the chunk reduction for small batches (few rows, many
// chunks): workgroup (tile, g) adds chunks g cpg .. (g + 1) cpg - 1 of its 64
// rows (its 4 waves interleaved, then in wave order) and stores the sum in
// chunk g cpg of the same buffer, which no other workgroup reads.
__global__ void __launch_bounds__(256) k_partial_reduce(double* __restrict__ partial, int n_chunks, int cpg, int nd,
                                                        int64_t n) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * 64 + lane;
  const int64_t pc = p < n ? p : n - 1;
  const int c0 = blockIdx.y * cpg;
  const int c1 = c0 + cpg < n_chunks ? c0 + cpg : n_chunks;
  double z[2 * kMaxDet];
#pragma unroll
  for (int j = 0; j < 2 * kMaxDet; ++j) z[j] = 0.0;
  for (int c = c0 + wave; c < c1; c += 4) {
#pragma unroll
    for (int j = 0; j < 2 * kMaxDet; ++j)
      if (j < 2 * nd) z[j] += partial[((int64_t)c * 2 * nd + j) * n + pc];
  }
  __shared__ double red[3][2 * kMaxDet][64];
  if (wave > 0) {
#pragma unroll
    for (int j = 0; j < 2 * kMaxDet; ++j) red[wave - 1][j][lane] = z[j];
  }
  __syncthreads();
  if (wave != 0 || p >= n) return;
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int j = 0; j < 2 * kMaxDet; ++j) z[j] += red[w][j][lane];
#pragma unroll
  for (int j = 0; j < 2 * kMaxDet; ++j)
    if (j < 2 * nd) partial[((int64_t)c0 * 2 * nd + j) * n + p] = z[j];
}

// Distance marginal: one lane per proposal, waves splitting the grid (see block_dist_lse).
// Small batches: one wave per proposal (see wave_dist_lse), which keeps many
// waves busy when there are few proposals.
template <int PREC>
__global__ void __launch_bounds__(256) k_dist_marg_w(const double* __restrict__ zbuf, int64_t n,
                                                     const double* __restrict__ tab, int n_dist, double dd,
                                                     const LogI0Consts* __restrict__ Cp, double* __restrict__ logl) {
  const LogI0Consts& C = *Cp;
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (p >= n) return;
  const double z1 = zbuf[p];
  const double hh1 = zbuf[n + p];
  if (z1 < 0.0) {
    if (lane == 0) logl[p] = -INFINITY;
    return;
  }
  const double v = PREC == 0 ? wave_dist_lse(z1, hh1, tab, n_dist, lane, C)
                             : wave_dist_lse_f32(z1, hh1, tab, n_dist, lane);
  if (lane == 0) logl[p] = -0.5 * dd + v;
}

// Large batches: a workgroup of kDistWaves waves per 64 proposals, the grid
// split between the waves (see block_dist_lse).
constexpr int kDistWaves = 16;
constexpr int64_t kDistSliced = 8192;  // batches from this size use the sliced form

template <int PREC>
__global__ void __launch_bounds__(1024) k_dist_marg(const double* __restrict__ zbuf, int64_t n,
                                                    const double* __restrict__ tab, int n_dist, double dd,
                                                    const LogI0Consts* __restrict__ Cp, double* __restrict__ logl) {
  const LogI0Consts& C = *Cp;
  __shared__ double red[kDistWaves * 64];
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 64 + lane;
  const int64_t pc = p < n ? p : n - 1;
  const double z1 = zbuf[pc];
  const double hh1 = zbuf[n + pc];
  // invalid rows (z1 < 0) still take part in the block's barriers
  const double v = block_dist_lse<PREC>(z1 < 0.0 ? 0.0 : z1, hh1, tab, n_dist, kDistWaves, red, C);
  if ((threadIdx.x >> 6) == 0 && p < n) logl[p] = z1 < 0.0 ? -INFINITY : -0.5 * dd + v;
}

// Materialise h_i(f_k) = A P_i f^(-7/6) exp(-2 pi i Phi_i(f)) for injections.
__global__ void __launch_bounds__(256) k_template(const double* __restrict__ coef, int64_t ld, int64_t n,
                                                  const double* __restrict__ bins, int rs, int nd, int64_t k0,
                                                  double df, int64_t n_freq, TrigConsts T,
                                                  double* __restrict__ h) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t p = blockIdx.y;
  if (k >= n_freq || p >= n) return;
  const bool valid = coef[C_VALID * ld + p] != 0.0;
  PhaseCoef c;
  c.a0 = coef[C_A0 * ld + p];
  c.a2 = coef[C_A2 * ld + p];
  c.a3 = coef[C_A3 * ld + p];
  c.a4 = coef[C_A4 * ld + p];
  c.a5 = coef[C_A5 * ld + p];
  c.a6 = coef[C_A6 * ld + p];
  c.a7 = coef[C_A7 * ld + p];
  c.a8 = coef[C_A8 * ld + p];
  c.a10 = coef[C_A10 * ld + p];
  c.a12 = coef[C_A12 * ld + p];
  c.b5 = coef[C_B5 * ld + p];
  c.b6 = coef[C_B6 * ld + p];
  const double* rec = bins + k * rs;
  const double r0 = phase_cycles(c, rec[0], rec[1], rec[2], rec[3]);
  const double f = (double)(k0 + k) * df;
  const double fa = pow(f, -7.0 / 6.0);
  for (int i = 0; i < nd; ++i) {
    const double dt = i == 0 ? 0.0 : coef[(C_DT1 + i - 1) * ld + p];
    double s, co;
    sincos_cycles(r0 + f * dt, T, &s, &co);
    const double ar = coef[(C_APRE + i) * ld + p] * fa;
    const double ai = coef[(C_APIM + i) * ld + p] * fa;
    // (ar + i ai) (co - i s)
    double* out = h + ((p * nd + i) * n_freq + k) * 2;
    out[0] = valid ? ar * co + ai * s : 0.0;
    out[1] = valid ? ai * co - ar * s : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Launch helpers

gw_status launch_prologue(gw_ctx* ctx, const double* theta, int64_t n, int marg, double* coef, int64_t ld,
                          hipStream_t st) {
  if (n == 0) return GW_OK;
  const int tpb = 256;
  const int64_t blocks = (n + tpb - 1) / tpb;
  hipLaunchKernelGGL(k_prologue, dim3((unsigned)blocks), dim3(tpb), 0, st, theta, n, marg, ctx->geom, coef, ld);
  return check_hip(hipGetLastError(), "prologue launch");
}

void full_launch_shape(const gw_ctx* ctx, int64_t n, int* tpb_out, int* chunks_out) {
  int tpb = ctx->full_tpb;
  int ch = ctx->full_chunks;
  if (tpb <= 0) tpb = n >= 2048 ? 256 : 64;
  const int64_t nptile = (n + tpb - 1) / tpb;
  if (ch <= 0) {
    // Aim for ~4096 workgroups of 4 waves (~2048 of 1), keep at least 32 bins
    // per chunk.  At 4096 x 259,585 with 4-wave workgroups, 256 chunks (16,384
    // waves) ran 12 % faster than 128: several waves per SIMD in flight, and a
    // short tail.
    const int64_t target = tpb >= 256 ? 4096 : 2048;
    int64_t want = (target + nptile - 1) / nptile;
    want = (want + 7) / 8 * 8;
    const int64_t maxc = ctx->geom.n_freq / 32 > 8 ? ctx->geom.n_freq / 32 : 8;
    if (want > maxc) want = maxc / 8 * 8 > 0 ? maxc / 8 * 8 : 8;
    if (want < 8) want = 8;
    ch = (int)want;
  }
  *tpb_out = tpb;
  *chunks_out = ch;
}

template <int ND>
static gw_status launch_full_nd(gw_ctx* ctx, const double* coef, int64_t ld, int64_t n, int prec, int tpb,
                                int n_chunks, double* partial, hipStream_t st) {
  const int nf = (int)ctx->geom.n_freq;
  const int chunk_len = (int)((nf + n_chunks - 1) / n_chunks);
  const TrigConsts T = make_trig_consts();
  const PhaseRuns PR = make_phase_runs(ctx->geom);
  const int64_t nptile = (n + tpb - 1) / tpb;
  const int64_t blocks = nptile * n_chunks;
  if (blocks > 0x7fffffff) return set_error(GW_EINVAL, "batch too large for one launch");
  if (prec == GW_PREC_FP64) {
    hipLaunchKernelGGL((k_full<ND, 0, false>), dim3((unsigned)blocks), dim3(tpb), 0, st, coef, ld, n, ctx->bins,
                       ctx->geom.k0, ctx->geom.df, nf, chunk_len, n_chunks, T, PR, 1.0, 0.0, nullptr, nullptr, partial);
  } else {
    hipLaunchKernelGGL((k_full<ND, 1, false>), dim3((unsigned)blocks), dim3(tpb), 0, st, coef, ld, n, ctx->bins,
                       ctx->geom.k0, ctx->geom.df, nf, chunk_len, n_chunks, T, PR, ctx->pgain_re, ctx->pgain_im,
                       nullptr, nullptr, partial);
  }
  return check_hip(hipGetLastError(), "full-band kernel launch");
}

template <int ND>
static gw_status launch_mfma_nd(gw_ctx* ctx, const double* coef, int64_t ld, int64_t n, int tpb, int n_chunks,
                                double* partial, hipStream_t st) {
  const int nf = (int)ctx->geom.n_freq;
  const int blk = ctx->mom_blk;
  const int per = (int)((nf + n_chunks - 1) / n_chunks);
  const int chunk_len = (per + blk - 1) / blk * blk;
  const int64_t nptile = (n + tpb - 1) / tpb;
  const int64_t blocks = nptile * n_chunks;
  if (blocks > 0x7fffffff) return set_error(GW_EINVAL, "batch too large for one launch");
  hipLaunchKernelGGL((k_full_mfma<ND>), dim3((unsigned)blocks), dim3(tpb), 0, st, coef, ld, n, ctx->bins,
                     ctx->wtab, ctx->geom.k0, ctx->geom.df, nf, (int)ctx->mom_pad, blk, chunk_len, n_chunks,
                     ctx->pgain_re, ctx->pgain_im, partial);
  return check_hip(hipGetLastError(), "full-band matrix-core kernel launch");
}

// Automatic choice: the vector-ALU reduction (measured faster at the
// benchmark shape); the matrix-core form on request.
bool use_mfma(const gw_ctx* ctx, int prec) {
  return prec == GW_PREC_MIXED && ctx->mom_blk > 0 && ctx->full_kernel == 2;
}

gw_status launch_full(gw_ctx* ctx, const double* coef, int64_t ld, int64_t n, int prec, int tpb, int n_chunks,
                      double* partial, hipStream_t st) {
  if (n == 0) return GW_OK;
  if (tpb != 64 && tpb != 128 && tpb != 256) return set_error(GW_EINVAL, "tpb must be 64, 128 or 256");
  if (n_chunks < 1) return set_error(GW_EINVAL, "n_chunks must be >= 1");
  if (ctx->full_kernel == 2 && prec == GW_PREC_MIXED && ctx->mom_blk == 0)
    return set_error(GW_ENOTSUP, "matrix-core reduction unavailable: detector delays too long for 8-bin blocks");
  if (use_mfma(ctx, prec)) {
    switch (ctx->n_det) {
      case 1: return launch_mfma_nd<1>(ctx, coef, ld, n, tpb, n_chunks, partial, st);
      case 2: return launch_mfma_nd<2>(ctx, coef, ld, n, tpb, n_chunks, partial, st);
      case 3: return launch_mfma_nd<3>(ctx, coef, ld, n, tpb, n_chunks, partial, st);
      case 4: return launch_mfma_nd<4>(ctx, coef, ld, n, tpb, n_chunks, partial, st);
      default: return set_error(GW_ENOTSUP, "n_det %d not supported", ctx->n_det);
    }
  }
  switch (ctx->n_det) {
    case 1: return launch_full_nd<1>(ctx, coef, ld, n, prec, tpb, n_chunks, partial, st);
    case 2: return launch_full_nd<2>(ctx, coef, ld, n, prec, tpb, n_chunks, partial, st);
    case 3: return launch_full_nd<3>(ctx, coef, ld, n, prec, tpb, n_chunks, partial, st);
    case 4: return launch_full_nd<4>(ctx, coef, ld, n, prec, tpb, n_chunks, partial, st);
    default: return set_error(GW_ENOTSUP, "n_det %d not supported", ctx->n_det);
  }
}

// Mean deviation of the FP32 hardware phasor g~ = cos(2 pi t) - i sin(2 pi t)
// from the exact one g over n uniform midpoints t in [-1/2, 1/2): per block,
// sum_i (g~_i conj(g_i) - 1), reduced in a fixed order.
__global__ void __launch_bounds__(256) k_phasor_bias(int n, TrigConsts T, double* __restrict__ out) {
  __shared__ double red[2][256];
  double ar = 0.0, ai = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float t = (float)(((double)i + 0.5) / (double)n - 0.5);
    const double c = (double)__builtin_amdgcn_cosf(t), sn = (double)__builtin_amdgcn_sinf(t);
    double se, ce;
    sincos_cycles((double)t, T, &se, &ce);
    // (c - i sn) (ce + i se)
    ar += c * ce + sn * se - 1.0;
    ai += c * se - sn * ce;
  }
  red[0][threadIdx.x] = ar;
  red[1][threadIdx.x] = ai;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = red[0][0];
    out[2 * blockIdx.x + 1] = red[1][0];
  }
}

gw_status calibrate_phasor(gw_ctx* ctx) {
  const int n = 1 << 20, blocks = 256;
  double* d = nullptr;
  gw_status s = check_hip(hipMalloc((void**)&d, 2 * blocks * sizeof(double)), "calibration buffer");
  if (s != GW_OK) return s;
  hipLaunchKernelGGL(k_phasor_bias, dim3(blocks), dim3(256), 0, nullptr, n, make_trig_consts(), d);
  std::vector<double> h(2 * blocks);
  s = check_hip(hipGetLastError(), "calibration launch");
  if (s == GW_OK) s = check_hip(hipMemcpy(h.data(), d, h.size() * sizeof(double), hipMemcpyDeviceToHost), "copy");
  (void)hipFree(d);
  if (s != GW_OK) return s;
  double br = 0.0, bi = 0.0;
  for (int b = 0; b < blocks; ++b) {
    br += h[2 * b];
    bi += h[2 * b + 1];
  }
  br /= n;
  bi /= n;
  // 1 / (1 + b)
  const double mr = 1.0 + br, m2 = mr * mr + bi * bi;
  ctx->pgain_re = mr / m2;
  ctx->pgain_im = -bi / m2;
  return GW_OK;
}

// Block length: the largest power of two B in [8, 256] with
// |phi| = pi df tau_max B small enough that the first dropped term of the
// rotation series, |phi|^KM / KM!, stays below 1e-9 (tau_max: the largest
// light travel time between detector 0 and another detector).
gw_status build_moment_table(gw_ctx* ctx, const std::vector<double>& rec, const double* det_pos) {
  const int nd = ctx->n_det;
  const int64_t nf = ctx->geom.n_freq;
  const double df = ctx->geom.df;
  const int km = nd > 1 ? (kMomCols - 1) / (nd - 1) : 0;
  double tau_max = 0.0;
  for (int i = 1; i < nd; ++i) {
    double d2 = 0.0;
    for (int j = 0; j < 3; ++j) {
      const double d = det_pos[3 * i + j] - det_pos[j];
      d2 += d * d;
    }
    tau_max = fmax(tau_max, sqrt(d2) / kLightSpeed);
  }
  double phi_max = 1e300;
  if (km > 0) {
    double fact = 1.0;
    for (int m = 2; m <= km; ++m) fact *= (double)m;
    phi_max = pow(1e-9 * fact, 1.0 / km);
  }
  int blk = 0;
  for (int b = 256; b >= 8; b >>= 1) {
    if (kPi * df * tau_max * b <= phi_max) {
      blk = b;
      break;
    }
  }
  ctx->mom_blk = 0;
  ctx->mom_pad = 0;
  if (blk == 0) return GW_OK;
  const int rs = 4 + 2 * nd;
  const int64_t npad = (nf + blk - 1) / blk * blk;
  std::vector<float> w((size_t)npad * 3 * kMomCols, 0.0f);
  const double cen = 0.5 * (blk - 1), half = 0.5 * blk;
  for (int64_t k = 0; k < nf; ++k) {
    const double t = ((double)(k % blk) - cen) / half;
    const double* r = &rec[(size_t)k * rs];
    float* wk = &w[(size_t)k * 3 * kMomCols];
    auto put = [&](int q, double ur, double ui) {
      wk[3 * q] = (float)ur;
      wk[3 * q + 1] = (float)(ui - ur);
      wk[3 * q + 2] = (float)(ur + ui);
    };
    put(0, r[4], r[5]);
    for (int i = 1; i < nd; ++i) {
      double tm = 1.0;
      for (int m = 0; m < km; ++m) {
        put(1 + (i - 1) * km + m, tm * r[4 + 2 * i], tm * r[5 + 2 * i]);
        tm *= t;
      }
    }
  }
  gw_status s = check_hip(hipMalloc((void**)&ctx->wtab, w.size() * sizeof(float)), "moment table alloc");
  if (s == GW_OK)
    s = check_hip(hipMemcpy(ctx->wtab, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice), "moment copy");
  if (s != GW_OK) return s;
  ctx->mom_blk = blk;
  ctx->mom_pad = npad;
  return GW_OK;
}

gw_status launch_epilogue(gw_ctx* ctx, double* partial, int n_chunks, const double* coef, int64_t ld,
                          int64_t n, int marg, int prec, double* logl, hipStream_t st) {
  return launch_epilogue_cached(ctx, partial, n_chunks, coef, ld, n, marg, prec, logl, nullptr, nullptr, nullptr, st);
}

gw_status launch_epilogue_cached(gw_ctx* ctx, double* partial, int n_chunks, const double* coef, int64_t ld,
                                 int64_t n, int marg, int prec, double* logl, const int32_t* zsrc, const double* zc,
                                 double* zrow, hipStream_t st) {
  return launch_epilogue_z(ctx, partial, n_chunks, coef, ld, n, marg, prec, logl, zsrc, zc, zrow, ctx->zbuf, st);
}

gw_status launch_epilogue_z(gw_ctx* ctx, double* partial, int n_chunks, const double* coef, int64_t ld, int64_t n,
                            int marg, int prec, double* logl, const int32_t* zsrc, const double* zc, double* zrow,
                            double* zbuf, hipStream_t st) {
  if (n == 0) return GW_OK;
  const int64_t blocks = (n + 63) / 64;
  const LogI0Consts* C = ctx->i0c;  // device copy, r1max from the distance grid
  int groups = n_chunks, cstride = 1;
  if (n <= 2048 && n_chunks >= 64) {
    // few rows, many chunks: reduce groups of 8 chunks across the chip first
    cstride = 8;
    groups = (n_chunks + cstride - 1) / cstride;
    hipLaunchKernelGGL(k_partial_reduce, dim3((unsigned)blocks, (unsigned)groups), dim3(256), 0, st, partial, n_chunks,
                       cstride, ctx->n_det, n);
    gw_status s = check_hip(hipGetLastError(), "partial reduction launch");
    if (s != GW_OK) return s;
  }
  hipLaunchKernelGGL(k_epilogue, dim3((unsigned)blocks), dim3(1024), 0, st, partial, groups, cstride, ctx->n_det, coef,
                     ld, n, ctx->dd, marg, logl, zbuf, zsrc, zc, zrow);
  gw_status s = check_hip(hipGetLastError(), "epilogue launch");
  if (s != GW_OK || marg != 2) return s;
  // large batches: lane = row (grid records are scalar loads shared by 64
  // rows); small batches: wave = row
  if (n >= kDistSliced) {
    const int64_t dblocks = (n + 63) / 64;
    if (prec == GW_PREC_MIXED)
      hipLaunchKernelGGL(k_dist_marg<1>, dim3((unsigned)dblocks), dim3(64 * kDistWaves), 0, st, zbuf, n,
                         ctx->dist_tab, ctx->n_dist, ctx->dd, C, logl);
    else
      hipLaunchKernelGGL(k_dist_marg<0>, dim3((unsigned)dblocks), dim3(64 * kDistWaves), 0, st, zbuf, n,
                         ctx->dist_tab, ctx->n_dist, ctx->dd, C, logl);
  } else {
    const int64_t dblocks = (n + 3) / 4;
    if (prec == GW_PREC_MIXED)
      hipLaunchKernelGGL(k_dist_marg_w<1>, dim3((unsigned)dblocks), dim3(256), 0, st, zbuf, n, ctx->dist_tab,
                         ctx->n_dist, ctx->dd, C, logl);
    else
      hipLaunchKernelGGL(k_dist_marg_w<0>, dim3((unsigned)dblocks), dim3(256), 0, st, zbuf, n, ctx->dist_tab,
                         ctx->n_dist, ctx->dd, C, logl);
  }
  return check_hip(hipGetLastError(), "distance marginal launch");
}

// Block length of the moment cache: the largest power of two B in [4, 512]
// with pi df B kTauCap <= 1.61.
int wmom_block(const gw_ctx* ctx) {
  int b = 4;
  while (b < 512 && kPi * ctx->geom.df * (2 * b) * kTauCap <= 1.61) b *= 2;
  return b;
}

int64_t wmom_slot_f2(const gw_ctx* ctx) {
  const int blk = wmom_block(ctx);
  const int64_t n_blk = (ctx->geom.n_freq + blk - 1) / blk;
  return n_blk * ctx->n_det * kWMom;
}

template <int ND>
static gw_status launch_cached_nd(gw_ctx* ctx, const double* coef, int64_t n, int prec, int tpb, int n_chunks,
                                  const int32_t* slow_rows, const int32_t* fast_rows, const int32_t* counts,
                                  int rows_per_slot, const int32_t* slot_of, const float2* mom, double* zfast,
                                  double* partial, hipStream_t st) {
  const int nf = (int)ctx->geom.n_freq;
  const TrigConsts T = make_trig_consts();
  const PhaseRuns PR = make_phase_runs(ctx->geom);
  const int64_t nptile = (n + 63) / 64;  // 64 rows per workgroup; tpb / 64 waves split each chunk
  const int64_t blocks = nptile * n_chunks;
  if (blocks > 0x7fffffff) return set_error(GW_EINVAL, "batch too large for one launch");
  const int chunk_len = (int)((nf + n_chunks - 1) / n_chunks);
  gw_status s = GW_OK;
  if (slow_rows) {
    if (prec == GW_PREC_FP64)
      hipLaunchKernelGGL((k_full<ND, 0, true>), dim3((unsigned)blocks), dim3(tpb), 0, st, coef, n, n, ctx->bins,
                         ctx->geom.k0, ctx->geom.df, nf, chunk_len, n_chunks, T, PR, 1.0, 0.0, slow_rows, counts, partial);
    else
      hipLaunchKernelGGL((k_full<ND, 1, true>), dim3((unsigned)blocks), dim3(tpb), 0, st, coef, n, n, ctx->bins,
                         ctx->geom.k0, ctx->geom.df, nf, chunk_len, n_chunks, T, PR, ctx->pgain_re, ctx->pgain_im,
                         slow_rows, counts, partial);
    s = check_hip(hipGetLastError(), "full-band list kernel launch");
  }
  if (s != GW_OK || !mom) return s;  // no cache, no fast rows
  const int blk = wmom_block(ctx);
  const int n_blk = (nf + blk - 1) / blk;
  // chunks of at least 8 blocks, at most the partials' chunk count
  int cm = n_blk / 8 < n_chunks ? n_blk / 8 : n_chunks;
  if (cm < 1) cm = 1;
  if (cm > 8) cm = cm / 8 * 8;
  const int slot = prof_begin(ctx, st, 1);
  hipLaunchKernelGGL((k_wmom<ND>), dim3((unsigned)(nptile * cm)), dim3(256), 0, st, coef, n, n, ctx->geom.k0,
                     ctx->geom.df, blk, n_blk, cm, zfast ? cm : n_chunks, T, fast_rows, counts + 1, rows_per_slot,
                     slot_of, mom, wmom_slot_f2(ctx), partial);
  prof_end(ctx, slot, st);
  s = check_hip(hipGetLastError(), "cached-waveform kernel launch");
  if (s != GW_OK || !zfast) return s;  // without zfast the epilogue sums the fast rows' partials
  hipLaunchKernelGGL(k_wmom_sum, dim3((unsigned)((n * 2 * ND + 255) / 256)), dim3(256), 0, st, partial, cm, ND, n,
                     fast_rows, counts + 1, zfast);
  return check_hip(hipGetLastError(), "cached-waveform sum launch");
}

gw_status launch_cached(gw_ctx* ctx, const double* coef, int64_t n, int prec, int tpb, int n_chunks,
                        const int32_t* slow_rows, const int32_t* fast_rows, const int32_t* counts, int rows_per_slot,
                        const int32_t* slot_of, const float2* mom, double* zfast, double* partial, hipStream_t st) {
  if (n == 0) return GW_OK;
  if (tpb != 64 && tpb != 128 && tpb != 256) return set_error(GW_EINVAL, "tpb must be 64, 128 or 256");
  switch (ctx->n_det) {
    case 1: return launch_cached_nd<1>(ctx, coef, n, prec, tpb, n_chunks, slow_rows, fast_rows, counts,
                                       rows_per_slot, slot_of, mom, zfast, partial, st);
    case 2: return launch_cached_nd<2>(ctx, coef, n, prec, tpb, n_chunks, slow_rows, fast_rows, counts,
                                       rows_per_slot, slot_of, mom, zfast, partial, st);
    case 3: return launch_cached_nd<3>(ctx, coef, n, prec, tpb, n_chunks, slow_rows, fast_rows, counts,
                                       rows_per_slot, slot_of, mom, zfast, partial, st);
    case 4: return launch_cached_nd<4>(ctx, coef, n, prec, tpb, n_chunks, slow_rows, fast_rows, counts,
                                       rows_per_slot, slot_of, mom, zfast, partial, st);
    default: return set_error(GW_ENOTSUP, "n_det %d not supported", ctx->n_det);
  }
}

template <int ND>
static void launch_wmom_build_nd(gw_ctx* ctx, const double* coef, int64_t ld, const int32_t* slots,
                                 const int32_t* count, int rows_per_slot, const int32_t* src, int prec, dim3 grid,
                                 float2* mom, hipStream_t st) {
  const int blk = wmom_block(ctx);
  const TrigConsts T = make_trig_consts();
  const PhaseRuns R = make_phase_runs(ctx->geom);
  if (prec == GW_PREC_FP64)
    hipLaunchKernelGGL((k_wmom_build<ND, 0>), grid, dim3(64), 0, st, coef, ld, slots, count, rows_per_slot, src,
                       ctx->bins, (int)ctx->geom.n_freq, blk, wmom_slot_f2(ctx), T, R, 1.0, 0.0,
                       (const double*)ctx->wc_basis, mom);
  else
    hipLaunchKernelGGL((k_wmom_build<ND, 1>), grid, dim3(64), 0, st, coef, ld, slots, count, rows_per_slot, src,
                       ctx->bins, (int)ctx->geom.n_freq, blk, wmom_slot_f2(ctx), T, R, ctx->pgain_re, ctx->pgain_im,
                       (const double*)ctx->wc_basis, mom);
}

gw_status launch_wmom_build(gw_ctx* ctx, const double* coef, int64_t ld, const int32_t* slots, const int32_t* count,
                            int64_t max_count, int rows_per_slot, const int32_t* src, int prec, float2* mom,
                            hipStream_t st) {
  if (max_count <= 0) return GW_OK;
  if (!ctx->wc_basis) return set_error(GW_ESTATE, "waveform cache: basis table missing");
  const int blk = wmom_block(ctx);
  const int n_blk = (int)((ctx->geom.n_freq + blk - 1) / blk);
  if (max_count < kWBuildManyRows) {
    // the sampler's rounds: cost follows the device-side count
    const TrigConsts T = make_trig_consts();
    const size_t lds = wmom_build_few_lds(blk, ctx->n_det);
    if (prec == GW_PREC_FP64)
      hipLaunchKernelGGL(k_wmom_build_few<0>, dim3(2048), dim3(256), lds, st, coef, ld, slots, count, rows_per_slot,
                         src, ctx->bins, ctx->rec_stride, (int)ctx->geom.n_freq, ctx->n_det, blk, n_blk,
                         wmom_slot_f2(ctx), T, 1.0, 0.0, (const double*)ctx->wc_basis, mom);
    else
      hipLaunchKernelGGL(k_wmom_build_few<1>, dim3(2048), dim3(256), lds, st, coef, ld, slots, count, rows_per_slot,
                         src, ctx->bins, ctx->rec_stride, (int)ctx->geom.n_freq, ctx->n_det, blk, n_blk,
                         wmom_slot_f2(ctx), T, ctx->pgain_re, ctx->pgain_im, (const double*)ctx->wc_basis, mom);
    return check_hip(hipGetLastError(), "waveform cache build launch");
  }
  const dim3 grid((unsigned)n_blk, (unsigned)((max_count + 63) / 64));
  switch (ctx->n_det) {
    case 1: launch_wmom_build_nd<1>(ctx, coef, ld, slots, count, rows_per_slot, src, prec, grid, mom, st); break;
    case 2: launch_wmom_build_nd<2>(ctx, coef, ld, slots, count, rows_per_slot, src, prec, grid, mom, st); break;
    case 3: launch_wmom_build_nd<3>(ctx, coef, ld, slots, count, rows_per_slot, src, prec, grid, mom, st); break;
    case 4: launch_wmom_build_nd<4>(ctx, coef, ld, slots, count, rows_per_slot, src, prec, grid, mom, st); break;
    default: return set_error(GW_ENOTSUP, "n_det %d not supported", ctx->n_det);
  }
  return check_hip(hipGetLastError(), "waveform cache build launch");
}

gw_status wmom_init(gw_ctx* ctx) {
  const int blk = wmom_block(ctx);
  std::vector<double> h((size_t)blk * kWMom);
  const double cen = 0.5 * (blk - 1), hinv = 2.0 / blk;
  for (int j = 0; j < blk; ++j) {
    // T_m of the bin's offset in the block, by the three-term recurrence
    const double t = ((double)j - cen) * hinv;
    double a = 1.0, b = t;
    for (int m = 0; m < kWMom; ++m) {
      h[(size_t)j * kWMom + m] = a;
      const double c = 2.0 * t * b - a;
      a = b;
      b = c;
    }
  }
  gw_status s = check_hip(hipMalloc((void**)&ctx->wc_basis, h.size() * sizeof(double)), "cache basis alloc");
  if (s == GW_OK)
    s = check_hip(hipMemcpy(ctx->wc_basis, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice),
                  "cache basis copy");
  return s;
}

gw_status launch_template(gw_ctx* ctx, const double* coef, int64_t ld, int64_t n, double* h, hipStream_t st) {
  if (n == 0) return GW_OK;
  if (n > 65535) return set_error(GW_EINVAL, "gw_template: at most 65535 rows per call");
  const int tpb = 256;
  const int64_t bx = (ctx->geom.n_freq + tpb - 1) / tpb;
  hipLaunchKernelGGL(k_template, dim3((unsigned)bx, (unsigned)n), dim3(tpb), 0, st, coef, ld, n, ctx->bins,
                     ctx->rec_stride, ctx->n_det, ctx->geom.k0, ctx->geom.df, ctx->geom.n_freq, make_trig_consts(), h);
  return check_hip(hipGetLastError(), "template launch");
}

}  // namespace gw

extern "C" gw_status gw_full_phase_runs(const gw_ctx* ctx, int32_t* k_min, int32_t* len) {
  if (!ctx) return gw::set_error(GW_EINVAL, "gw_full_phase_runs: ctx is NULL");
  const gw::PhaseRuns R = gw::make_phase_runs(ctx->geom);
  for (int j = 0; j < 4; ++j) {
    if (k_min) k_min[j] = R.k_min[j];
    if (len) len[j] = R.len[j];
  }
  return GW_OK;
}
