// Host-side definition of the library context and the internal launch
// helpers shared by the library's HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "gw_device.h"
#include "gwswig.h"

struct gw_het_state;
struct gw_graph_cache;
struct gw_slice_ws;

struct gw_ctx {
  int device = 0;
  gw::Geom geom{};
  int n_det = 0;
  double dd = 0.0;                 // sum_i <d_i|d_i>
  // full-band per-bin records [n_freq][4 + 2 n_det] FP64:
  //   x = f^(1/3), x^2, f^(-5/3), ln f, then Re/Im of u_ik per detector
  double* bins = nullptr;
  int rec_stride = 0;
  // distance grid
  double* dist_tab = nullptr;      // [n_dist][4]: d, 1/d, 1/(2 d^2), ln w
  int32_t n_dist = 0;
  double dist_r1max = 0.0;         // max_j 1/d_j
  std::vector<double> h_dist_grid, h_dist_logw;
  // host copies kept for heterodyne set-up
  std::vector<double> h_data_re, h_data_im, h_psd;
  // device copy of the ln I0 coefficients (r1max set from the distance grid),
  // for kernels that read them through a pointer
  gw::LogI0Consts* i0c = nullptr;
  // workspace (grown on demand)
  double* coef = nullptr;          // [C_NCOEF][cap_n]
  int64_t coef_cap = 0;
  double* partial = nullptr;       // full-band partial sums
  int64_t partial_cap = 0;         // doubles
  double* zbuf = nullptr;          // [2][cap_n] (|Z1|, <h|h>_1) for the distance marginal
  int64_t zbuf_cap = 0;
  // launch configuration of the full-band kernel (0 = heuristic)
  int full_tpb = 0;
  int full_chunks = 0;
  int full_kernel = 0;             // 0 auto, 1 vector-ALU reduction, 2 matrix-core reduction (mixed only)
  // 1 / (1 + b), b the mean complex deviation of the FP32 hardware phasor
  // cos(2 pi t) - i sin(2 pi t) from the exact one over uniform t (measured at
  // context creation); applied to the mixed reductions' sums
  double pgain_re = 1.0, pgain_im = 0.0;
  // matrix-core form of the mixed reduction: block moments
  //   W[k][q][plane], q = detector/moment column, planes (w_r, w_i - w_r, w_r + w_i)
  float* wtab = nullptr;
  int mom_blk = 0;                 // bins per block (power of two, >= 8); 0 = form unavailable
  int64_t mom_pad = 0;             // n_freq rounded up to a multiple of mom_blk
  // kernel timing (gw_profile_enable / gw_profile_read)
  int prof = 0;                     // 0 off, 1 the dominant kernel, 2 the time-grid kernel
  std::vector<hipEvent_t> prof_ev;  // pairs (start, stop)
  int prof_used = 0;
  // time marginal: window half-width (s), FFT twiddles and moment workspace
  double tm_window = 0.1;
  int tm_R = 4;                    // grid points per sampling interval of the segment
  int tm_nsk = 0;                  // edge chunks of the heterodyned time marginal's moments (0 = heuristic)
  double* wc_basis = nullptr;      // [wmom_block][12] Chebyshev values for the waveform cache
  double* tm_ccoef = nullptr;      // [K][256][16] expansion coefficients of the grid (tm_cc_L, tm_cc_jmax, tm_cc_K)
  int tm_cc_L = 0, tm_cc_jmax = 0, tm_cc_K = 0;
  double* tm_basis = nullptr;      // [blk][K] Chebyshev values of the in-block offset for the moments
  int tm_basis_blk = 0, tm_basis_K = 0;
  double* tm_mom = nullptr;
  int64_t tm_mom_cap = 0;
  // bumped by every setter that changes what a captured likelihood launch
  // holds as arguments (grid shapes, launch shapes, heterodyne state)
  uint64_t gen = 0;
  // sampler sky frame: 0 equatorial (ra, dec), 1 zenith and azimuth about the
  // baseline of detectors sky_a -> sky_b; sky_det_time: coordinate 10 is the
  // arrival time at detector sky_a
  int sky_frame = 0, sky_a = 0, sky_b = 1, sky_det_time = 0;
  // post-hoc reconstruction workspace: (Re Z, Im Z, <h|h>) [3][n], per-detector
  // sums [n][2 n_det], log L [n]
  double* recon = nullptr;
  int64_t recon_cap = 0;
  gw_het_state* het = nullptr;
  gw_graph_cache* graphs = nullptr;
  gw_slice_ws* slice = nullptr;
};

namespace gw {

gw_status set_error(gw_status st, const char* fmt, ...);
gw_status check_hip(hipError_t e, const char* what);
gw_status ensure_buffer(double** buf, int64_t* cap, int64_t need, const char* what);

// Launch helpers (all asynchronous on ``st``).
gw_status launch_prologue(gw_ctx* ctx, const double* theta, int64_t n, int marg, double* coef,
                          int64_t ld, hipStream_t st);
gw_status launch_full(gw_ctx* ctx, const double* coef, int64_t ld, int64_t n, int prec,
                      int tpb, int n_chunks, double* partial, hipStream_t st);
// The partials may be overwritten (small batches reduce them in place first).
gw_status launch_epilogue(gw_ctx* ctx, double* partial, int n_chunks, const double* coef,
                          int64_t ld, int64_t n, int marg, int prec, double* logl, hipStream_t st);
gw_status launch_template(gw_ctx* ctx, const double* coef, int64_t ld, int64_t n, double* h,
                          hipStream_t st);
// Waveform-cache forms (fast/slow blocks of the sampler).  A cache slot holds
// the block moments of one intrinsic waveform (float2 [n_blk][n_det][12],
// wmom_slot_f2 entries; block length wmom_block bins).  launch_cached runs the
// full reduction on rows slow_rows[0 .. counts[0]) (none when slow_rows is
// NULL) into partials of n_chunks chunks and row stride n (coefficients with
// ld = n), and, when mom is not NULL, the moment reduction on rows
// fast_rows[0 .. counts[1]) (row p uses slot slot_of[p], or p / rows_per_slot
// when slot_of is NULL), whose complete sums go to zfast[p][2 n_det] (rows
// whose |t_c + dt_i| exceeds the cache's range get NaN), or, when zfast is
// NULL, into the same n_chunks partials as the full reduction (summed by the
// epilogue like any other row).
// launch_epilogue_cached combines partials (rows with zsrc[p] >= 0 take their
// sums from zc[zsrc[p]]) and writes every row's sums to zrow when not NULL.
// launch_wmom_build rebuilds the slots slots[i] >= 0, i < *count <= max_count,
// from coefficient row src[i] (slot * rows_per_slot when src is NULL), with
// the phase and phasor of precision prec.
int wmom_block(const gw_ctx* ctx);
int64_t wmom_slot_f2(const gw_ctx* ctx);
gw_status launch_cached(gw_ctx* ctx, const double* coef, int64_t n, int prec, int tpb, int n_chunks,
                        const int32_t* slow_rows, const int32_t* fast_rows, const int32_t* counts, int rows_per_slot,
                        const int32_t* slot_of, const float2* mom, double* zfast, double* partial, hipStream_t st);
gw_status launch_epilogue_cached(gw_ctx* ctx, double* partial, int n_chunks, const double* coef, int64_t ld,
                                 int64_t n, int marg, int prec, double* logl, const int32_t* zsrc, const double* zc,
                                 double* zrow, hipStream_t st);
// As launch_epilogue_cached, with the distance marginal's (|Z_1|, <h|h>_1)
// staging buffer [2][n] given explicitly instead of the context's.
gw_status launch_epilogue_z(gw_ctx* ctx, double* partial, int n_chunks, const double* coef, int64_t ld, int64_t n,
                            int marg, int prec, double* logl, const int32_t* zsrc, const double* zc, double* zrow,
                            double* zbuf, hipStream_t st);
gw_status launch_wmom_build(gw_ctx* ctx, const double* coef, int64_t ld, const int32_t* slots, const int32_t* count,
                            int64_t max_count, int rows_per_slot, const int32_t* src, int prec, float2* mom,
                            hipStream_t st);
// The cache's Chebyshev table [wmom_block][12] (built at context creation).
gw_status wmom_init(gw_ctx* ctx);
// Cached-likelihood launch shape (64 rows per workgroup, chunks of ~512 bins)
// and the workspace it needs for n rows.
void cached_shape(const gw_ctx* ctx, int* tpb, int* nch);
gw_status cached_reserve(gw_ctx* ctx, int64_t n);
void full_launch_shape(const gw_ctx* ctx, int64_t n, int* tpb, int* n_chunks);
// Block-moment table of the matrix-core reduction from the per-bin records
// (host [n_freq][4 + 2 n_det]); leaves the form unavailable (mom_blk = 0) when
// the detector delays are too long for a block of 8 bins.
gw_status build_moment_table(gw_ctx* ctx, const std::vector<double>& rec, const double* det_pos);
// Measure the hardware phasor bias and set ctx->pgain_re / pgain_im.
gw_status calibrate_phasor(gw_ctx* ctx);

// Time-grid sums from block moments (gw_tgrid.hip), shared by the full-band
// and heterodyned time marginals: moments [n][K][n_blk] complex (K expansion
// orders, 12 or 16), one FFT of length L = P R per order, the grid
// t_j = j delta / R, |j| <= jmax.
constexpr int kTgHMax = 48;  // most norm moments of the heterodyned form
struct TGridArgs {
  const double* mom;   // complex moment (row p, order m, block b) at p rs + (m n_blk + b) es
  int64_t mom_rs, mom_es;  // (K n_blk, 1): row-major, one row's moments contiguous; (1, n): row fastest
  int64_t n;
  int n_blk, L, jmax, K;
  const double* coef;  // prologue coefficients of the n rows (stride ld)
  int64_t ld;
  double* logl;
  int het;             // heterodyned norm: hhc [n], hpart [n_hch][n][mh] complex
  const double* hhc;
  const double* hpart;
  int n_hch, mh;
  double hw_step;      // 2 pi hw / (N R)
  int64_t c2, cden;    // exp(-2 pi i c u_j) = exp(-2 pi i (c2 j mod cden) / cden)
  double* zout;        // or NULL: [n][2 jmax + 1][3] staged grid values
  double f0_num, f0_den;  // f_0 t_j = j f0_num / f0_den cycles
  double* zpart;       // [tgrid_split(n, K)][n][2 jmax + 1] complex when the split exceeds 1
};
// The context's time grid: segment length N (samples), J and R (|j| <= jmax =
// J R), P, blocks of blk = N / P fine bins (n_blk of them), L = P R.
struct TimeGridShape {
  int64_t N;
  double delta;  // the segment's sampling interval; the grid step is delta / R
  int J, R, P, blk, n_blk, L, jmax;
};
gw_status time_grid_shape(const gw_ctx* ctx, TimeGridShape* g);
// The context's coefficient table for a grid (rebuilt when L, jmax or K
// change), and the rows per chunk whose moments fit the bounded workspace.
gw_status tgrid_tables(gw_ctx* ctx, int L, int jmax, int K);
int64_t tgrid_chunk_rows(int64_t n, int n_blk, int K);
// Order groups per row of a launch of n rows (1, 2 or 4); above 1 the launch
// needs zpart.
int tgrid_split(int64_t n, int K);
// Complex elements of zpart needed by the launches of n rows in chunks of
// chunk rows on a grid of nt points.
int64_t tgrid_zpart_elems(int64_t n, int64_t chunk, int K, int nt);
gw_status launch_tgrid(const gw_ctx* ctx, const TGridArgs& a, hipStream_t st);

// Record the device address of ``device``'s copy of the allocation-free
// workspace (gw_noalloc.hip); called by gw_ctx_create with the device
// current, once per device.
gw_status noalloc_init(int device);

// Prescreen network hooks for the sampler (gw_mlp.hip): the context a
// network was made on; a counter that changes whenever its input/output
// scaling changes (a captured inference launch bakes the scaling in);
// refreshing the BF16 weight copies (not inside a capture); the BF16
// inference of n unit-cube rows x [n][11] into out [n] (log L units).
const gw_ctx* mlp_ctx(const gw_mlp* m);
uint64_t mlp_scale_version(const gw_mlp* m);
gw_status mlp_prepare(gw_mlp* m, hipStream_t st);
gw_status mlp_infer(gw_mlp* m, const double* x, int64_t n, double* out, hipStream_t st);

// Kernel timing: record a start / stop event pair around the dominant kernel.
// prof_begin returns the pair index or -1 when timing is off or full.
int prof_begin(gw_ctx* ctx, hipStream_t st, int which = 1);
void prof_end(gw_ctx* ctx, int slot, hipStream_t st);

// Grow the workspace a likelihood call of n rows needs, without launching
// (graph capture must not allocate); het_shape_key reports the heterodyned
// launch shape (zeros without heterodyne set-up).
gw_status full_reserve(gw_ctx* ctx, int64_t n);
gw_status het_reserve(gw_ctx* ctx, int64_t n);
// Write the argument block of the single batch (theta, n rows, logl) now, on
// st; until het_unpin_args or a call with other arguments, heterodyned calls
// on that batch launch no argument kernel (a sampler's rounds, graph-captured
// or not, reuse the block).  The caller keeps other calls off the context
// meanwhile.
gw_status het_pin_args(gw_ctx* ctx, const double* theta, int64_t n, double* logl, hipStream_t st);
void het_unpin_args(gw_ctx* ctx);
void het_shape_key(const gw_ctx* ctx, int32_t* wpb, int32_t* grid, int32_t* ech);
// The heterodyned time marginal's table and index addresses and plan sizes
// (zeros without heterodyne state), for keying captured graphs.
void het_tm_key(const gw_ctx* ctx, const void** tab, const void** idx, int32_t* nch, int32_t* nslot, int32_t* nsplit);

// Heterodyne and graph state owned by the context.
void het_free(gw_ctx* ctx);
void graphs_free(gw_ctx* ctx);
void slice_free(gw_ctx* ctx);
gw_status loglike_het(gw_ctx* ctx, const double* theta, int64_t n, int marg, int prec, double* logl,
                      hipStream_t st);
// Heterodyned likelihood that also stages each row's (Re Z, Im Z, <h|h>) in
// zc3 [3][n] (Re Z NaN for rows that are not physical).
gw_status loglike_het_staged(gw_ctx* ctx, const double* theta, int64_t n, int marg, int prec, double* logl,
                             double* zc3, hipStream_t st);
// Any likelihood (like, marg = GW_MARG_PHASE or GW_MARG_PHASE_DIST, prec):
// stage each row's (Re Z, Im Z, <h|h>) in ctx->recon [3][n] and its log L in
// logl (NULL: in the work space).
gw_status stage_overlaps(gw_ctx* ctx, const double* theta, int64_t n, int like, int marg, int prec, double* logl,
                         hipStream_t st);
// Full-band phase+time marginal (GW_MARG_PHASE_TIME).
gw_status loglike_tmarg(gw_ctx* ctx, const double* theta, int64_t n, int prec, double* logl, hipStream_t st);
// Phase+time marginals that also stage each row's grid values for post-hoc
// draws: zout [n][N_t][3] = (Re Z(t_j), Im Z(t_j), <h|h>(t_j)), Re NaN for
// unphysical rows.
gw_status loglike_tmarg_staged(gw_ctx* ctx, const double* theta, int64_t n, int prec, double* logl, double* zout,
                               hipStream_t st);
gw_status loglike_het_tmarg_staged(gw_ctx* ctx, const double* theta, int64_t n, int prec, double* logl,
                                   double* zout, hipStream_t st);
// Build the tables and size the work space a phase+time marginal of n rows
// uses (like GW_FULL or GW_HET), launching nothing: afterwards such a call
// allocates nothing and can be captured into a graph.
gw_status tmarg_reserve(gw_ctx* ctx, int64_t n, int like);

}  // namespace gw
