/*
 * gwswig.h - C ABI of the batched gravitational-wave likelihood library
 * (libgwswig.so, HIP for gfx950).
 *
 * The library evaluates the matched-filter log-likelihood of the paper's
 * Sec. III.A, Eq. (loglike),
 *     log L(theta) = -1/2 sum_i <d_i - h_i(theta) | d_i - h_i(theta)>_i,
 *     <a|b>_i      = 4 Re int a*(f) b(f) / S_i(f) df,
 * for a batch of parameter vectors at once, with the analytic phase and
 * distance marginalisations of Sec. III.A, on the full uniform frequency grid
 * or on the heterodyned (relative-binning) grid of Sec. III.D.  The template
 * is a TaylorF2 aligned-spin tidal inspiral (a stand-in for the paper's
 * waveform family) projected on each detector through its antenna pattern
 * and time delay.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 * - Parameter vectors are FP64, 13 columns, row-major [n, 13]:
 *     Mc (Msun, detector frame), q = m2/m1 in (0, 1], chi1, chi2, Lambda1,
 *     Lambda2, d_L (Mpc), iota, ra, dec, psi, phi_c, t_c (s).
 *   Modes that marginalise phi_c (and d_L) ignore those columns.
 * - Frequency grid: f_k = (k0 + k) * df, k = 0 .. n_freq - 1 (both band
 *   edges included); the inner product is the Riemann sum over that grid.
 * - Device buffers are caller-owned, contiguous, and must stay alive until
 *   the work queued on the caller's stream has completed.  The context owns
 *   everything it uploads.  A context is not thread-safe; all work goes on the
 *   stream passed in (a hipStream_t, NULL for the default stream).  A context
 *   serves one stream at a time: its workspaces (coefficients, partial sums,
 *   marginal buffers) are shared by every call, so two calls on one context
 *   queued on different streams race unless the caller orders them (finish
 *   one stream's work, or make the second stream wait on an event recorded
 *   after the first call).  Use one context per stream for concurrent work.
 * - Errors are returned as status codes; nothing throws across the ABI and on
 *   an error no output is written.  gw_last_error() returns a thread-local
 *   message for the last non-OK status of the calling thread.
 * - A parameter vector that is non-finite or unphysical (Mc <= 0, q outside
 *   (0, 1], |chi| >= 1, d_L <= 0 where d_L is used) gets log L = -inf; it is
 *   not an error, so one bad row never fails a batch.
 * - Asynchronous device faults surface at the next synchronising call.
 */
#ifndef GWSWIG_H
#define GWSWIG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gw_ctx gw_ctx;
typedef struct gw_mlp gw_mlp;  /* prescreen network, see gw_mlp_create */

typedef enum {
  GW_OK = 0,
  GW_EINVAL = -1,   /* bad argument (null pointer, size, mode) */
  GW_ENOMEM = -2,   /* device or host allocation failed */
  GW_EDEVICE = -3,  /* HIP runtime error or no usable device */
  GW_ESTATE = -4,   /* call not valid in the context's current state */
  GW_ENOTSUP = -5   /* unsupported configuration */
} gw_status;

/* Likelihood kind. */
enum { GW_FULL = 0, GW_HET = 1 };
/* Marginalisation (Sec. III.A and the appendix on grid marginals): none,
 * phi_c, phi_c and d_L, phi_c and t_c (loglike_batch only; see
 * gw_set_time_window). */
enum { GW_MARG_NONE = 0, GW_MARG_PHASE = 1, GW_MARG_PHASE_DIST = 2, GW_MARG_PHASE_TIME = 3 };
/* Arithmetic: plain FP64, or FP64 phase with FP32 phasors and sums. */
enum { GW_PREC_FP64 = 0, GW_PREC_MIXED = 1 };

#define GW_MAX_DET 4
#define GW_NPARAM 13

/*
 * Problem description (host pointers, FP64; copied at gw_ctx_create, the
 * caller keeps ownership).  Cited definitions: strain d_i(f) and one-sided
 * PSD S_i(f) of Sec. III.A; distance prior proportional to d_L^2 on a 1-D
 * grid (Sec. III.A).
 *   n_det        number of detectors, 1 .. GW_MAX_DET
 *   k0, n_freq   grid start index and number of bins (n_freq >= 1)
 *   df           bin width (Hz), > 0
 *   data_re/im   [n_det, n_freq] real and imaginary parts of d_i(f_k)
 *   psd          [n_det, n_freq] S_i(f_k) > 0
 *   det_tensor   [n_det, 3, 3] detector response tensors (Earth-fixed frame)
 *   det_pos      [n_det, 3] detector positions (m, Earth-fixed frame)
 *   gmst         Greenwich sidereal angle (rad); phi = ra - gmst
 *   dist_grid    [n_dist] d_L grid (Mpc), > 0; may be NULL if n_dist == 0
 *   dist_logw    [n_dist] log prior-times-quadrature weights of the grid
 */
typedef struct {
  int32_t n_det;
  int64_t k0;
  int64_t n_freq;
  double df;
  const double* data_re;
  const double* data_im;
  const double* psd;
  const double* det_tensor;
  const double* det_pos;
  double gmst;
  const double* dist_grid;
  const double* dist_logw;
  int32_t n_dist;
} gw_problem;

/* Message of the calling thread's last non-OK status ("" if none). */
const char* gw_last_error(void);

/* Library version string. */
const char* gw_version(void);

/*
 * Create a context on HIP device ``device``: uploads the weighted data
 * u_ik = 4 df d_ik* f_k^(-7/6) / S_ik, the per-bin frequency tables, the
 * closed-form template-norm weights W_i = 4 df sum_k f_k^(-7/3) / S_ik and
 * <d|d>.  *out receives the context (NULL on error).
 * Errors: GW_EINVAL (null pointers, bad sizes, non-positive PSD or df),
 * GW_EDEVICE (no device), GW_ENOMEM.
 */
gw_status gw_ctx_create(const gw_problem* problem, int32_t device, gw_ctx** out);

/* Release every device buffer of the context; NULL is accepted. */
gw_status gw_ctx_destroy(gw_ctx* ctx);

/* sum_i <d_i|d_i> held by the context (host FP64). */
gw_status gw_data_inner(const gw_ctx* ctx, double* dd_out);

/*
 * Batched log-likelihood (Sec. III.A, Eq. loglike; marginalisations of
 * Sec. III.A; heterodyned form of Sec. III.D when like == GW_HET).
 *   theta   device [n, 13] FP64 parameter vectors
 *   n       batch size (0 is a no-op)
 *   like    GW_FULL or GW_HET (GW_HET needs heterodyne_setup first)
 *   marg    GW_MARG_NONE, GW_MARG_PHASE, GW_MARG_PHASE_DIST or
 *           GW_MARG_PHASE_TIME
 *   prec    GW_PREC_FP64 or GW_PREC_MIXED
 *   logl    device [n] FP64 output
 *   stream  hipStream_t or NULL
 * Errors: GW_EINVAL, GW_ESTATE (heterodyne not set up, or PHASE_DIST with an
 * empty distance grid), GW_EDEVICE, GW_ENOMEM.
 */
gw_status loglike_batch(gw_ctx* ctx, const double* theta, int64_t n, int32_t like,
                        int32_t marg, int32_t prec, double* logl, void* stream);

/*
 * Coalescence-time marginal (GW_MARG_PHASE_TIME, with the phase marginal;
 * the appendix's grid sum over time shifts, evaluated by FFT on the uniform
 * grid).  The t_c column of theta is ignored; d_L is used.  On the grid
 * t_j = j delta / R, |j| <= J R, J = floor(W / delta), delta = 1 / (N df) with N
 * the smallest power of two >= 2 (k0 + n_freq - 1) (the segment's sampling
 * interval) and R the oversampling (gw_set_time_oversample, default 4: the
 * paper's dense grid; on the plain interval the sum of I0(|Z|) misses the
 * integral by tens of nats for loud signals):
 *   log L = -<d|d>/2 - <h|h>/2 + ln[ (1/N_t) sum_j I0(|Z(t_j)|) ],
 * Z(t) the overlap of the template shifted by t (template at t_c = 0).  The
 * library cuts the band into blocks of N / P bins (P the smallest power of two
 * >= 2 J + 1, and at least 16 / R), within which the time shift is expanded in
 * Chebyshev polynomials of the bin's offset (Jacobi-Anger: K = 12 terms when
 * the dropped ones stay below 2e-11 of the block's sum of |overlap weight|,
 * every grid of the default window, else 16), and evaluates every grid point
 * with one FFT of length P R per term over the blocks.  W defaults to 0.1 s;
 * gw_set_time_window changes it (GW_ENOTSUP if P would exceed 2048); a grid
 * whose transform P R would exceed 4096 points is GW_ENOTSUP at evaluation.
 * gw_time_grid_info reports the grid step delta / R, the number of points
 * N_t = 2 J R + 1, P and the block length.  Work space: n x (n_freq / B) x
 * 16 K bytes per call (in row chunks of at most 1 GiB).
 * With like = GW_HET the same grid sum runs on the binned likelihood, the
 * appendix's direct summation on the heterodyned bins: at every t_j the
 * phase-marginal binned log L of the template shifted by t_j (the binned
 * <h|h> depends on t_j through the bin widths).  The library forms per-row
 * edge weights, takes their block moments (the edges lie on the fine grid) into
 * the same FFTs as the full band, and expands the bin-width phasors
 * exp(-2 pi i (f_e - f_e-1) t_j) about the widths' centre (as many terms as
 * keep the first dropped one below 1e-13 of the norm sum; GW_ENOTSUP beyond
 * 48).  Work space up to 1 GiB of moments per chunk of rows (about 8,000 rows
 * at 128 s).
 */
gw_status gw_set_time_window(gw_ctx* ctx, double window);
/* Grid points per sampling interval of the time marginal: 1, 2, 4 (default),
 * 8 or 16; GW_EINVAL otherwise.  Applies from the next call on. */
gw_status gw_set_time_oversample(gw_ctx* ctx, int32_t factor);
gw_status gw_time_grid_info(const gw_ctx* ctx, double* delta, int32_t* n_points, int32_t* fft_len,
                            int32_t* block_bins);

/*
 * Post-hoc reconstruction of the marginalised distance and phase (appendix on
 * grid marginalisations: the marginalised parameters of each posterior sample
 * are drawn after the run from their exact conditional on the grid, computed
 * from the sample's inner products).  For each row of theta (device [n, 13],
 * as for loglike_batch with the same like, marg and prec; phi_c ignored, d_L
 * ignored for GW_MARG_PHASE_DIST), with Z, <h|h> the sample's overlap and norm
 * at phi_c = 0 (at d_L = 1 Mpc for the distance marginal):
 *   marg = GW_MARG_PHASE_DIST: d_L = d_j drawn from the grid weights
 *       exp(ln w_j - <h|h>_1 / (2 d_j^2) + ln I0(|Z_1| / d_j)), then
 *       phi_c given d_j;
 *   marg = GW_MARG_PHASE: d_L = the sample's own, phi_c drawn;
 *   marg = GW_MARG_PHASE_TIME (d_L sampled, t_c ignored): t_c = t_j drawn on
 *       the time grid of the marginal (see gw_set_time_window) from the
 *       weights exp(-<h|h>(t_j)/2 + ln I0(|Z(t_j)|)), Z(t_j) the overlap of the
 *       template shifted by t_j, then phi_c given t_j with Z' = Z(t_j);
 *       out[p][0] is then t_c (s) and idx[p][0] the grid index j (t_j =
 *       (j - J) delta);
 *   phi_c = 2 pi m / n_phase drawn from the weights
 *       exp(kappa cos(2 pi m / n_phase + arg Z')), Z' = Z / d_L, kappa = |Z'|
 *       (the template carries exp(+i phi_c)).
 * Each draw takes the first grid index whose cumulative weight exceeds
 * u times the total weight, with u from ``uniforms`` (device [n, 2]:
 * distance, phase; each in (0, 1)).
 * out:    device [n, 2] (d_L in Mpc, phi_c in rad).
 * idx:    device [n, 2] (distance-grid index or -1, phase index) or NULL.
 * logl:   device [n] the row's marginal log L (as loglike_batch), or NULL.
 * Unphysical rows give NaN and indices -1.  n_phase: 1 .. 2^20 (2048 is a
 * good default: the conditional has width 1 / sqrt(kappa)).  Errors:
 * GW_ENOTSUP for GW_MARG_NONE, GW_ESTATE without a distance grid (distance
 * marginal) or heterodyne set-up (like = GW_HET).  Work space grows to
 * n (4 + 2 n_det) doubles, or n (3 N_t + 1) for the time marginal; the
 * context's likelihood work space is reused.
 */
gw_status gw_reconstruct(gw_ctx* ctx, const double* theta, int64_t n, int32_t like, int32_t marg, int32_t prec,
                         const double* uniforms, int32_t n_phase, double* out, int32_t* idx, double* logl,
                         void* stream);

/*
 * Projected templates h_i(f_k) on the full grid (Sec. III.A): one parameter
 * vector per row of ``theta`` (device [n, 13]); ``h`` is device
 * [n, n_det, n_freq, 2] FP64 (interleaved real, imaginary).  Rows that are
 * unphysical are written as zeros.  Used to build injections.
 */
gw_status gw_template(gw_ctx* ctx, const double* theta, int64_t n, double* h, void* stream);

/*
 * Allocation-free full-band likelihood, for callers that cannot allocate
 * device memory (work recorded into a graph, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, kernels and results as
 * loglike_batch with like = GW_FULL, for marg GW_MARG_NONE, GW_MARG_PHASE or
 * GW_MARG_PHASE_DIST; nothing is allocated: the per-row coefficients, the
 * distance marginal's staging and the frequency-chunk partial sums live in
 * one static device array of GW_NOALLOC_DOUBLES FP64 values (16 MiB) per
 * device, held from the first context created on that device until the
 * process ends.  A row needs C + 2 + 2 n_det c doubles for c frequency
 * chunks (C = 32 coefficients); the launch shape's chunk count is lowered in
 * steps of 8 (at least 8) until the batch fits, so results agree with
 * loglike_batch up to summation order, and bit for bit when both run the same
 * shape (gw_set_full_shape).  Every call on a device shares that device's
 * array: calls that overlap on one device (other streams, threads or
 * contexts) race, and the caller must order them.
 * Errors: GW_EINVAL (n above floor(GW_NOALLOC_DOUBLES / (34 + 16 n_det)),
 * 25,575 rows at 3 detectors; a fixed launch shape that does not fit; a bad
 * mode), GW_ESTATE (PHASE_DIST without a distance grid), GW_EDEVICE.
 */
#define GW_NOALLOC_DOUBLES (1 << 21)
gw_status loglike_batch_noalloc(gw_ctx* ctx, const double* theta, int64_t n, int32_t marg, int32_t prec,
                                double* logl, void* stream);

/*
 * Heterodyne (relative-binning) set-up, Sec. III.D: builds the bin grid of
 * "equal maximum phase change" shared across the network and the
 * per-detector summary data of the reference template h0 = h(theta0).
 *   theta0     host [13] reference parameters (must be physical)
 *   n_bins     requested bins, 1 .. n_freq - 1; edges are snapped to the
 *              fine grid and merged, so the context may hold fewer (see
 *              gw_het_info)
 *   bin_rule   0: equal steps of the phase bound
 *                 sum_g sgn(g) (f / f*_g)^g, g in {-5/3, -2/3, 1, 5/3, 7/3},
 *                 f*_g = f_max for g > 0 else f_min;
 *              1: geometric (log-spaced) edges
 *   edges_out  host [n_bins + 1] edge frequencies (Hz), or NULL; only the
 *              first (held bins + 1) entries are written
 * Replaces any previous summary data and drops captured graphs.  Blocks
 * until the set-up has completed.  Errors: GW_EINVAL, GW_EDEVICE, GW_ENOMEM.
 */
gw_status heterodyne_setup(gw_ctx* ctx, const double* theta0, int32_t n_bins, int32_t bin_rule,
                           double* edges_out);

/* Number of bins held after heterodyne_setup.  GW_ESTATE before set-up. */
gw_status gw_het_info(const gw_ctx* ctx, int32_t* n_bins);

/*
 * Batched log-likelihood over uneven sub-batches in one launch sequence
 * (persistent work-list kernels; with use_graph != 0 the sequence is
 * captured once per (marg, prec, launch shape) into a hipGraph and replayed).
 *   theta     device [n_rows, 13]
 *   subs      device int64 [2 * n_sub]: (row offset, row count) pairs; rows
 *             outside [0, n_rows) are clipped, counts <= 0 are empty
 *   n_sub     number of sub-batches, 0 .. 65536
 *   like      GW_HET (the full-band form returns GW_ENOTSUP)
 *   logl      device [n_rows]; only rows covered by a sub-batch are written
 * The work list is read on the device, so one captured graph serves every
 * sub-batch layout.  Errors as loglike_batch.
 */
gw_status loglike_batch_uneven(gw_ctx* ctx, const double* theta, int64_t n_rows, const int64_t* subs,
                               int32_t n_sub, int32_t like, int32_t marg, int32_t prec, int32_t use_graph,
                               double* logl, void* stream);

/* Launch shape of the heterodyned kernels: waves per workgroup (1, 2, 4),
 * persistent grid size in workgroups and number of edge chunks a row's bins
 * are split into (0 = heuristic for either). */
gw_status gw_set_het_shape(gw_ctx* ctx, int32_t waves_per_block, int32_t grid, int32_t n_ech);
/* Edge chunks of the heterodyned time marginal's per-row edge moments (App. A
 * on the binned likelihood): 1, 2, 4, ..., 256 asks for that many edge
 * ranges of about equal cost (an edge or a frequency block one unit; a block
 * cut by several ranges gets its moments summed from their pieces in order;
 * fewer ranges when there are fewer units), 0 (default) restores the
 * heuristic (about 4096 (row tile, chunk) waves, at most 256 chunks of at
 * least 8 units).  Results differ only by summation order.  GW_EINVAL
 * otherwise. */
gw_status gw_set_het_tm_split(gw_ctx* ctx, int32_t n_chunks);

/* Number of instantiated graphs and the last instantiation time (ms), which
 * plays the role of a one-off compilation cost. */
gw_status gw_graph_info(const gw_ctx* ctx, int32_t* n_graphs, double* last_instantiate_ms);

/*
 * Constrained slice step (Sec. II.B Eq. cprior, Sec. II.C Eq. block_cprior,
 * Sec. III.B): one hit-and-run slice update of one Gibbs block for each of k
 * chains on the constrained prior pi(theta) 1[log L(theta) > log L*].
 * The sampler space is the 11-dimensional unit cube
 *   [Mc, q, chi1, chi2, Lambda1, Lambda2, iota, ra, dec, psi, t_c]
 * of the uniform / isotropic prior Mc in [1.1, 1.4], q in [0.5, 1],
 * chi in [-0.05, 0.05], Lambda in [0, 5000], cos(iota) and sin(dec)
 * uniform, ra in [0, 2 pi), psi in [0, pi), t_c in [-0.1, 0.1] s, with phi_c
 * and d_L marginalised (marg = GW_MARG_PHASE_DIST), or, with marg =
 * GW_MARG_PHASE_TIME (the paper's GW170817 configuration), phi_c and t_c
 * marginalised and d_L sampled as coordinate 10 in place of t_c (see
 * gw_prior_transform_marg).
 * A block holds 1 .. GW_MAX_BLOCK coordinates; one holding all 11 is the
 * unblocked nested slice sampler of the sampler-configuration section.
 * With F = GW_SLICE_UNI_FIXED(block_dim) = max(4, 2 ceil(block_dim / 2)) + 2:
 * per chain, u a uniform unit vector (Box-Muller pair p from uniforms 2p and
 * 2p + 1, the first block_dim normals, normalised), the direction d = L u
 * with L the block's lower Cholesky factor; a bracket [-r w, (1 - r) w] with
 * r = uniform F - 2; each end stepped out by w while log L > log L*, the
 * stepping-out budget m = 2 max_out + 1 split by V = uniform F - 1 into at
 * most J = floor(m V) steps for the lower end and m - 1 - J for the upper
 * one (Neal 2003, Sec. 4.1: a split drawn at random keeps the move
 * reversible when a cap binds); then shrink draws
 * t = t_lo + u_s (t_hi - t_lo), s = 0 .. max_shrink - 1 (uniform F + s),
 * until log L > log L*, the bracket end on the side of t moving to t.  A point
 * outside the cube fails without a likelihood call.  After max_shrink
 * failures the chain keeps its point (status 1).
 * Random numbers: ``uniforms`` (device [k, F + max_shrink]) when not NULL,
 * else Philox4x64-10 (Salmon et al. 2011): uniform j of chain c is word j % 4
 * of the block at counter (counter, c, j / 4, 0) under key (seed, 0), mapped
 * to ((w >> 11) + 0.5) 2^-53.
 * Blocks until done (the host checks progress every four rounds; rounds
 * after every chain has finished change nothing).
 */
#define GW_MAX_BLOCK 11
#define GW_SLICE_UNI_FIXED(bd) (((bd) <= 4 ? 4 : 2 * (((bd) + 1) / 2)) + 2)

typedef struct {
  int64_t k;              /* number of chains */
  double* x;              /* device [k, 11] unit-cube points, updated in place */
  double* logl;           /* device [k] log L of x, updated in place */
  double logl_star;       /* constraint log L* */
  const int32_t* block;   /* host [block_dim] coordinate indices 0..10, distinct */
  int32_t block_dim;      /* 1 .. GW_MAX_BLOCK */
  const double* chol;     /* host [block_dim, block_dim] lower-triangular, row-major */
  uint64_t seed;          /* Philox key */
  uint64_t counter;       /* Philox counter base */
  const double* uniforms; /* device [k, F + max_shrink] or NULL */
  double w;               /* bracket width along t (> 0) */
  int32_t max_out;        /* 0 .. 10000: half the stepping-out budget */
  int32_t max_shrink;     /* 1 .. 10000 */
  int32_t like;           /* GW_FULL or GW_HET */
  int32_t marg;           /* GW_MARG_PHASE_DIST */
  int32_t prec;           /* GW_PREC_FP64 or GW_PREC_MIXED */
  int32_t* n_evals;       /* device [k] likelihood calls per chain, or NULL */
  int32_t* status;        /* device [k] 0 moved, 1 kept, or NULL */
  int32_t use_graph;      /* 1: replay a captured graph of 4 rounds (captured on
                             first use and again when k, like, marg, prec, the
                             launch shapes, the time grid (window, oversampling,
                             edge split), the heterodyne setup, a workspace,
                             the network or its scaling change); 0: launch each
                             kernel.  Results are identical. */
  gw_mlp* mlp;            /* learned prescreen (a network made on this context)
                             or NULL: see below */
  double margin;          /* with mlp: finite; candidates predicted
                             >= log L* - margin get their exact log L */
  double audit_frac;      /* with mlp: in [0, 1], the share of the other
                             candidates evaluated anyway (audit) */
  int64_t* screen_stats;  /* host [3] or NULL: candidates screened out,
                             audited, audited and inside log L > log L* (a
                             false negative of the screen); synchronises */
  double* rec_x;          /* device [rec_cap, 11] or NULL: every exactly
                             evaluated candidate's unit-cube point goes to
                             slot (*rec_count)++ mod rec_cap (the pairs the
                             sampler generates, for training the prescreen);
                             slots are claimed in no fixed order */
  double* rec_logl;       /* device [rec_cap]: its exact log L */
  int64_t rec_cap;        /* >= 1 with rec_x */
  unsigned long long* rec_count;  /* device counter, set by the caller */
} gw_slice_args;

/*
 * Learned prescreen inside the slice update (spec learned form; the
 * paper's sampler evaluates every candidate).  With mlp, every round runs the
 * network on each candidate's unit-cube point (BF16 matrix-core inference,
 * FP32 accumulation; the prediction is compared in FP64).  A candidate whose
 * prediction is >= log L* - margin gets its exact log L (like, marg, prec);
 * otherwise it is taken as outside the constraint without a likelihood call
 * (a stepping-out end stops there, a shrink draw shrinks the bracket), unless
 * it is drawn for the audit: test ``idx`` of kind ``kind`` (0 lower end, 1
 * upper end, 2 shrink draw; idx counts that kind's tests in the block) of
 * chain c in block b is audited when word 0 of Philox4x64-10 at counter
 * (counter + b, c, kind, idx) under key (seed, 1), mapped as the uniforms
 * above, is below audit_frac; an audited candidate gets its exact log L and
 * that value decides.  Every accepted point therefore carries an exact log L;
 * a screened-out candidate that lies inside the constraint (a false
 * negative) shortens the bracket, which the audit counts.  n_evals counts
 * exact evaluations only.  The network's input scaling and weights are read
 * at each call; the same network may not be trained concurrently.
 * Errors: GW_EINVAL (network from another context, non-finite margin,
 * audit_frac outside [0, 1]).
 */
gw_status slice_step(gw_ctx* ctx, const gw_slice_args* args, void* stream);

/*
 * One Gibbs sweep (Sec. II.C Eq. block_cprior, Sec. III.B): every chain
 * applies the slice update above to blocks 0 .. n_blocks - 1 in order, block b
 * drawing its uniforms from Philox counter (counter + b, c, j / 4, 0).  Each
 * chain's result is bit-for-bit that of n_blocks successive slice_step calls
 * with counters counter, counter + 1, ... (same k, like, marg, prec and launch
 * shapes), but a chain starts its next block as soon as it has finished one,
 * so a sweep takes about the largest per-chain total of rounds instead of the
 * sum over blocks of the largest per-block count.  The explicit uniforms
 * table is not available here.  n_evals sums the likelihood calls over the
 * sweep; status counts the blocks whose shrink cap was hit.
 */
typedef struct {
  int64_t k;               /* number of chains */
  double* x;               /* device [k, 11], updated in place */
  double* logl;            /* device [k], updated in place */
  double logl_star;        /* constraint log L* */
  int32_t n_blocks;        /* 1 .. 16 */
  const int32_t* block_dim;/* host [n_blocks], each 1 .. GW_MAX_BLOCK */
  const int32_t* block;    /* host [n_blocks, GW_MAX_BLOCK] coordinate indices,
                              the first block_dim[b] of row b used, distinct,
                              0 .. 10 */
  const double* chol;      /* host [n_blocks, GW_MAX_BLOCK, GW_MAX_BLOCK] lower
                              Cholesky factor of each block, row-major, leading
                              block_dim[b] rows and columns used.  The
                              distinct blocks (a block equal to an earlier one
                              in coordinates and factor is not distinct) may
                              hold at most 160 factor entries (block_dim^2
                              each); beyond that GW_EINVAL. */
  uint64_t seed;           /* Philox key */
  uint64_t counter;        /* counter base of block 0 */
  double w;                /* bracket width along t (> 0) */
  int32_t max_out;         /* 0 .. 10000, as for slice_step */
  int32_t max_shrink;      /* 1 .. 10000 */
  int32_t like;            /* GW_FULL or GW_HET */
  int32_t marg;            /* GW_MARG_PHASE_DIST */
  int32_t prec;            /* GW_PREC_FP64 or GW_PREC_MIXED */
  int32_t* n_evals;        /* device [k] likelihood calls per chain, or NULL */
  int32_t* status;         /* device [k] blocks kept at the shrink cap, or NULL */
  int32_t use_graph;       /* as for slice_step */
  int32_t use_cache;       /* 1 (like = GW_FULL only): fast/slow waveform
                              cache, below */
  int64_t* eval_kinds;     /* host [3] or NULL: with the cache, likelihood
                              evaluations of the sweep in full (waveform
                              generated, seeding included), from the cached
                              waveform, and from the cached sums; -1 each
                              without the cache.  Synchronises the stream. */
  gw_mlp* mlp;             /* learned prescreen or NULL, as for slice_step */
  double margin;           /* as for slice_step */
  double audit_frac;       /* as for slice_step */
  int64_t* screen_stats;   /* as for slice_step (summed over the sweep) */
  double* rec_x;           /* as for slice_step */
  double* rec_logl;
  int64_t rec_cap;
  unsigned long long* rec_count;
} gw_sweep_args;

gw_status slice_sweep(gw_ctx* ctx, const gw_sweep_args* args, void* stream);
/*
 * Waveform cache (Sec. III.B: slow blocks regenerate the waveform, fast
 * blocks reuse a cached one and only redo the projection).  With use_cache a
 * block whose coordinates are all among {iota, psi} is projection-only: its
 * candidates reuse the overlaps z_i of the chain's current point and cost
 * O(1); a block among {iota, ra, dec, psi, t_c} is extrinsic: its candidates
 * reuse the chain's cached waveform, held as block moments (see
 * gw_wcache_loglike, kind 1), and only the detector delays change; any other
 * block evaluates in full (prec as given).  Each sweep first evaluates every
 * chain's current point in full to seed the overlaps (k extra evaluations,
 * not counted in n_evals).  A chain's waveform is rebuilt lazily: when it is
 * in an extrinsic block after a slow move (or at the start of the sweep), that
 * round's candidates evaluate in full and the rebuild follows the round.
 * Device memory: k x (n_freq / B) x n_det x 16 x 8 bytes (B the moment block,
 * 256 bins at df = 1/128 Hz), at most 64 GiB, kept with the context.  Results
 * agree with use_cache = 0 to rounding, so a near tie with log L* can resolve
 * differently.
 */

/*
 * The sampler's prior transform: unit-cube points x (device [n, 11], layout
 * as for slice_step) to parameter vectors theta (device [n, 13]; d_L = 1 and
 * phi_c = 0, both marginalised).  Used to evaluate a fresh live set.
 */
gw_status gw_prior_transform(gw_ctx* ctx, const double* x, int64_t n, double* theta, void* stream);
/* The same for a sampler run with marg = GW_MARG_PHASE_DIST (as above) or
 * GW_MARG_PHASE_TIME: then coordinate 10 is d_L, with a prior proportional to
 * d_L^2 between the first and last distance-grid nodes (inverse CDF
 * d = (d_1^3 + u (d_n^3 - d_1^3))^(1/3)), and t_c = 0 (marginalised). */
gw_status gw_prior_transform_marg(gw_ctx* ctx, const double* x, int64_t n, int32_t marg, double* theta,
                                  void* stream);

/*
 * Sky frame of the sampler's unit cube (blocked-kernel section: the source
 * direction is sampled as zenith and azimuth about a detector baseline rather
 * than as (ra, dec); the same section suggests detector-frame time too).
 * frame = 0: coordinates 7 and 8 are ra and dec (the default).  frame = 1:
 * with n = (r_b - r_a) / |r_b - r_a| the baseline of detectors det_a and
 * det_b (Earth-fixed positions), e1 the Earth's axis z made orthogonal to n
 * (x when |n_z| > 0.99) and e2 = n x e1, coordinate 7 is the azimuth
 * kappa = 2 pi u_7 and coordinate 8 the zenith acos(1 - 2 u_8), so that
 * s = cos(zen) n + sin(zen) (cos(kappa) e1 + sin(kappa) e2), dec = asin(s_z),
 * ra = atan2(s_y, s_x) + gmst (mod 2 pi).  Uniform points give an isotropic
 * sky, as before; the delay between the two detectors depends on the zenith
 * alone.  det_time = 1 (frame 1 only, not with GW_MARG_PHASE_TIME): coordinate
 * 10 is the arrival time t_a at detector det_a, uniform on [-0.1, 0.1] s, and
 * t_c = t_a + s . r_a / c (the geocentre t_c is then uniform only away from
 * the ends of its range).  Applies to slice_step, slice_sweep and the prior
 * transforms from the next call on.  GW_EINVAL for bad detectors or flags.
 */
gw_status gw_set_sky_frame(gw_ctx* ctx, int32_t frame, int32_t det_a, int32_t det_b, int32_t det_time);

/*
 * Maximum-likelihood search for the heterodyne fiducial (GW170817 section:
 * the reference parameters of the relative binning come from a
 * maximum-likelihood optimisation over priors narrowed to the event; the
 * limitations section notes that a deployment has to find them).  Maximises
 * the full-band phase+distance marginal log L (like = GW_FULL,
 * marg = GW_MARG_PHASE_DIST, the given prec) over the box [lo, hi] of the
 * sampler's unit cube (in the context's sky frame) by differential evolution,
 * DE/rand/1/bin (Storn & Price 1997): in generation g, member i draws
 * uniforms u_j = Philox4x64-10 word j % 4 of counter (g, i, j / 4, 0) under
 * key (seed, 2), mapped to ((w >> 11) + 0.5) 2^-53; u_0, u_1, u_2 choose three
 * distinct partners r1, r2, r3 other than i (r1 the floor(u_0 (P - 1))-th
 * index of 0..P-1 without i, r2 the floor(u_1 (P - 2))-th without {i, r1},
 * r3 the floor(u_2 (P - 3))-th without {i, r1, r2}); coordinate j takes the
 * mutant x_r1 + F (x_r2 - x_r3) (computed without fused multiply-add) when
 * j = floor(11 u_3) or u_(4+j) < CR, else x_ij; a mutant coordinate outside
 * [lo_j, hi_j] is mirrored at the wall it crossed and clipped.  All trials of
 * a generation are made first; a trial then replaces its member when its
 * log L is not NaN and at least the member's (or the member's is NaN).
 * x:          device [pop, 11] initial population inside the box, replaced by
 *             the final population.
 * fx:         device [pop] log L of the final population.
 * theta_best: host [13] parameter vector of the best member, with d_L and
 *             phi_c at the peak of the unmarginalised likelihood:
 *             phi_c = -arg Z_1 (mod 2 pi) and d_L = <h|h>_1 / |Z_1|, from the
 *             member's FP64 overlap Z_1 and norm <h|h>_1 at d_L = 1 Mpc.
 * Synchronises the stream.  Work space pop x 25 doubles for the call.
 * Errors: GW_EINVAL for pop outside 4 .. 2^22, generations < 0, F outside
 * (0, 2], CR outside [0, 1], a box outside [0, 1]; GW_ESTATE without a
 * distance grid; GW_EDEVICE when no member has a finite log L or the best
 * one has no overlap with the data.
 */
typedef struct {
  int64_t pop;            /* population size P */
  int32_t generations;    /* >= 0 */
  double f_scale;         /* F */
  double cr;              /* CR */
  uint64_t seed;          /* Philox key word 0 */
  const double* lo;       /* host [11] or NULL (zeros) */
  const double* hi;       /* host [11] or NULL (ones) */
  int32_t prec;           /* GW_PREC_FP64 or GW_PREC_MIXED */
} gw_fiducial_args;

gw_status gw_fiducial_search(gw_ctx* ctx, const gw_fiducial_args* args, double* x, double* fx, double* theta_best,
                             void* stream);

/*
 * Waveform cache (Sec. III.B, Sec. III.A): the slow / fast likelihood pair.
 * A slot holds one point's overlaps z_i = sum_k u_ik exp(-2 pi i Phi_ik)
 * and its intrinsic waveform g_k = exp(-2 pi i Psi(f_k)) (Psi the TaylorF2
 * phase without the linear time term) as block moments: for blocks of B bins
 * with centre f_c and t_j = (j - (B - 1)/2) / (B/2),
 *     M_m = sum_j t_j^m u_ij g_j,   m < 16   (FP64 sums stored as FP32),
 * so that a delay tau_i contributes
 *     exp(-2 pi i f_c tau_i) sum_m (-i pi df B tau_i)^m / m! M_m
 * per block.  B is the largest power of two up to 512 with
 * pi df B 0.25 s <= 1.61 (256 at df = 1/128 Hz), which keeps the first
 * dropped term below 1e-10 of the block's sum of |u g| for |tau_i| <= 0.25 s.
 *
 * gw_wcache_update (slow): full-band log L of theta (device [n, 13]; marg,
 *   prec as for loglike_batch) into logl (device [n]), and row r's overlaps
 *   and moments into slot slots[r] (device int32 [n]).  When a slot appears
 *   more than once the largest row index wins; a slot outside 0 .. n_slots-1
 *   stores nothing and gives log L = NaN.
 * gw_wcache_loglike (fast): log L of rows that differ from the point of
 *   their slot slots[r] only in extrinsic parameters, without generating a
 *   waveform:
 *     kind 1: ra, dec, psi, iota, t_c (and d_L) may differ; the moments are
 *             summed with each detector's delay t_c + dt_i (16 terms per
 *             block, FP64 arithmetic); rows with |t_c + dt_i| > 0.25 s get
 *             NaN;
 *     kind 2: only psi, iota (and d_L) may differ; the cached overlaps are
 *             reprojected, O(1) per row.
 *   Intrinsic parameters (Mc, q, chi1, chi2, Lambda1, Lambda2) and, for
 *   marg = GW_MARG_NONE, phi_c must equal the slot's; nothing checks this.
 *   Slots outside 0 .. n_slots-1 give log L = NaN.
 * Device memory: n_slots x (n_freq / B) x n_det x 128 bytes (at most
 * 128 GiB) plus the overlaps.  Errors as loglike_batch; GW_EINVAL for kind
 * not 1 or 2.
 */
typedef struct gw_wcache gw_wcache;
gw_status gw_wcache_create(gw_ctx* ctx, int64_t n_slots, gw_wcache** out);
gw_status gw_wcache_destroy(gw_wcache* cache);
gw_status gw_wcache_update(gw_wcache* cache, const double* theta, const int32_t* slots, int64_t n, int32_t marg,
                           int32_t prec, double* logl, void* stream);
gw_status gw_wcache_loglike(gw_wcache* cache, const double* theta, const int32_t* slots, int64_t n, int32_t kind,
                            int32_t marg, int32_t prec, double* logl, void* stream);

/*
 * Learned prescreen (not part of the paper's method, which uses exact
 * likelihoods only): a network 11 -> 256 -> 256 -> 256 -> 1 with exact GELU
 * g(z) = z Phi(z), inputs the standardised unit-cube point of gw_slice_args,
 * output the standardised log L.  Weights W_l are [fan_in, fan_out] row-major
 * followed by the bias, layers in order (134,913 FP32 values, gw_mlp_n_params).
 * Training is mean squared error with Adam (b1 0.9, b2 0.999, eps 1e-8) in
 * FP32; inference runs the hidden layers with BF16 weights and activations on
 * the matrix cores, accumulated in FP32.
 */
/* He-normal weights from ``seed``, zero biases; identity scaling. */
gw_status gw_mlp_create(gw_ctx* ctx, uint64_t seed, gw_mlp** out);
gw_status gw_mlp_destroy(gw_mlp* mlp);
gw_status gw_mlp_n_params(int64_t* n);
/* Input standardisation (x - x_mean) / x_std per coordinate (host [11]) and
 * output scaling log L = y_mean + y_std * y. */
gw_status gw_mlp_set_scaling(gw_mlp* mlp, const double* x_mean, const double* x_std, double y_mean, double y_std);
/* Host FP32 parameter vector in the layout above; set resets Adam's state. */
gw_status gw_mlp_set_params(gw_mlp* mlp, const float* params);
gw_status gw_mlp_get_params(gw_mlp* mlp, float* params);
/* Gradients of the mean squared error on (x device [n, 11], logl device [n])
 * into host [n_params]; the loss (standardised units) into *loss when not
 * NULL.  Synchronises the stream. */
gw_status gw_mlp_grad(gw_mlp* mlp, const double* x, const double* logl, int64_t n, float* grads, float* loss,
                      void* stream);
/* One Adam step of learning rate ``lr`` on a batch; *loss (before the step)
 * when not NULL (then synchronises). */
gw_status gw_mlp_train_step(gw_mlp* mlp, const double* x, const double* logl, int64_t n, float lr, float* loss,
                            void* stream);
/* Predicted log L for x (device [n, 11]) into out (device [n]); use_bf16
 * selects the matrix-core path, else the FP32 path. */
gw_status gw_mlp_forward(gw_mlp* mlp, const double* x, int64_t n, double* out, int32_t use_bf16, void* stream);

/*
 * Prescreened exact evaluation of candidate points x (device [n, 11], unit
 * cube as for gw_slice_args; phi_c and d_L marginalised).  With use_mlp the
 * network predicts log L for every candidate (BF16 path); candidates with a
 * prediction >= logl_star - margin, plus an audit fraction of the others
 * (Philox4x64-10 word 0 of counter (i, 0, 0, 0), key (seed, 1), below
 * audit_frac), get the exact likelihood (like, prec); without use_mlp every
 * candidate does.  logl (device [n]) receives the exact value or -inf for a
 * candidate not evaluated; flags (device int32 [n]) bit0 evaluated exactly,
 * bit1 predicted to pass, bit2 audited; pred (device [n] or NULL) the
 * predictions; *n_exact the number of exact evaluations.  An accept decision
 * must use logl only.  Synchronises the stream once (to size the exact batch).
 */
gw_status gw_prescreen_batch(gw_ctx* ctx, gw_mlp* mlp, const double* x, int64_t n, double logl_star, double margin,
                             double audit_frac, uint64_t seed, int32_t use_mlp, int32_t like, int32_t prec,
                             double* logl, double* pred, int32_t* flags, int64_t* n_exact, void* stream);

/*
 * Autotuner: times every candidate launch shape of the full-band (like =
 * GW_FULL) or heterodyned (GW_HET) kernels on the caller's batch ``theta``
 * (device [n, 13]), ``reps`` timed calls each after one warm-up, keeps the
 * fastest in the context and returns it: best_shape[0..2] = (proposals per
 * workgroup, frequency chunks, 0) for the full band or (waves per workgroup,
 * persistent workgroups, edge chunks with 0 = heuristic) for the heterodyned
 * form; *best_ms the mean time of one call.  Synchronises the stream.  Errors
 * as loglike_batch.
 */
gw_status gw_autotune(gw_ctx* ctx, const double* theta, int64_t n, int32_t like, int32_t marg, int32_t prec,
                      int32_t reps, int32_t* best_shape, double* best_ms, void* stream);

/*
 * Launch shape of the full-band kernel: ``tpb`` proposals per workgroup (64,
 * 128 or 256, i.e. 1, 2 or 4 waves walking the same frequency chunk) and
 * ``n_chunks`` frequency chunks (a multiple of 8 keeps every chunk on one
 * XCD).  0 restores the built-in heuristic.  Used by the
 * autotuner; results do not depend on the shape beyond summation order.
 */
gw_status gw_set_full_shape(gw_ctx* ctx, int32_t tpb, int32_t n_chunks);

/*
 * Reduction used by the mixed-precision full band: 0 automatic (currently the
 * vector-ALU form, the faster one at a batch of 4096), 1 vector ALUs (one sin/cos per bin, per-detector delay
 * rotation by recurrence), 2 matrix cores (block moments: the delay rotation
 * of detectors 1.. is expanded within blocks of B bins in powers of the bin
 * offset, truncated where the first dropped term is below 1e-9, and the block
 * moments are an FP32 contraction on v_mfma_f32_16x16x4_f32, folded into FP64
 * per block).  Kind 2 on a context where the form is unavailable makes
 * loglike_batch return GW_ENOTSUP.  The FP64 form always uses kind 1.
 */
gw_status gw_set_full_kernel(gw_ctx* ctx, int32_t kind);
/* Block length B of the matrix-core form (0 when the detectors are too far
 * apart for a block of 8 bins at this frequency spacing). */
gw_status gw_full_info(const gw_ctx* ctx, int32_t* mom_blk);
/*
 * Phase recurrence of the vector-ALU mixed reduction.  The TaylorF2 phase
 * (Sec. III.A) is evaluated over runs of bins: bin k lies in the run
 * [s, s + len[j] - 1], s = k rounded down to a multiple of len[j], for the
 * first level j (0..3; len descending powers of two) with s >= k_min[j], and
 * in no run (phase evaluated directly) if there is none.  A run evaluates the
 * phase directly on its top four bins and continues downwards with a cubic
 * finite-difference recurrence, three additions per bin; the levels keep the
 * recurrence's extrapolation error below 2e-8 cycles for chirp masses down
 * to 0.8 Msun.  A bin's phase depends only on its run, so results do not
 * depend on the launch shape beyond summation order.  Fills four entries of
 * each non-NULL output.  The FP64 form evaluates every bin directly.
 */
gw_status gw_full_phase_runs(const gw_ctx* ctx, int32_t* k_min, int32_t* len);

/*
 * Correction factor 1 / (1 + b) applied to the mixed full-band sums, where b
 * is the mean complex deviation g~ conj(g) - 1 of the FP32 hardware phasor
 * g~ = cos(2 pi t) - i sin(2 pi t) from the exact one over 2^20 uniform
 * arguments t, measured once at gw_ctx_create.  Every full-band sum is linear
 * in the phasor, so removing the mean bias leaves only the unbiased rounding,
 * whose effect on log L averages down over the bins.
 */
gw_status gw_phasor_gain(const gw_ctx* ctx, double* re, double* im);

/*
 * Kernel timing for roofline reporting.  enable = 1: the dominant kernel (the
 * full-band overlap kernel, the heterodyned evaluation kernel, or the moment
 * kernel of a time marginal); enable = 2: the time-grid kernel of the time
 * marginals; 0 turns timing off.  While enabled, every launch of the chosen
 * kernel is bracketed by HIP events recorded on the launch stream.
 * gw_profile_read waits for the recorded events, returns the summed kernel
 * time (ms) and the number of launches, and clears the record.  At most 4096
 * launches are recorded between reads (later ones are not timed).
 */
gw_status gw_profile_enable(gw_ctx* ctx, int32_t enable);
gw_status gw_profile_read(gw_ctx* ctx, double* kernel_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* GWSWIG_H */
