"""MI355X (gfx950) batched gravitational-wave likelihood for slice-within-Gibbs
nested sampling.

The compute lives in ``libgwswig.so`` (hand-written HIP); this package only
marshals arguments to its C ABI (``_lib``) and wraps the context in a small
class.  There is no CPU fallback: importing works without the library, but
every call that needs it raises if it has not been built.
"""
from . import _lib  # noqa: F401
from ._lib import (  # noqa: F401
    GW_FULL, GW_HET, GW_MARG_NONE, GW_MARG_PHASE, GW_MARG_PHASE_DIST, GW_MARG_PHASE_TIME, GW_PREC_FP64, GW_PREC_MIXED,
    GwError, gw_ctx_create, gw_ctx_destroy, gw_data_inner, gw_last_error, gw_set_full_shape, gw_template,
    gw_version, loglike_batch, heterodyne_setup, gw_het_info, loglike_batch_uneven, gw_set_het_shape,
    gw_graph_info, gw_profile_enable, gw_profile_read, slice_step, slice_sweep, gw_prior_transform, Mlp,
    gw_set_full_kernel, gw_full_info, gw_full_phase_runs, gw_phasor_gain, WaveformCache, gw_set_time_window,
    gw_time_grid_info, gw_set_het_tm_split, gw_reconstruct, slice_uniforms_fixed, GW_MAX_BLOCK, gw_set_sky_frame,
    gw_fiducial_search, gw_set_time_oversample, loglike_batch_noalloc, noalloc_max_rows, GW_NOALLOC_DOUBLES,
)


class Context:
    """Owns one library context (problem data resident on one GPU)."""

    def __init__(self, prob, device: int = 0):
        self.n_det = int(prob.data.shape[0])
        self.n_freq = int(prob.n_freq)
        self.device = device
        self._ctx = gw_ctx_create(prob, device)

    @property
    def handle(self):
        return self._ctx

    def loglike(self, theta, like=GW_FULL, marg=GW_MARG_NONE, prec=GW_PREC_FP64, out=None, stream=None):
        return loglike_batch(self._ctx, theta, like, marg, prec, out, stream)

    def template(self, theta, stream=None):
        return gw_template(self._ctx, theta, self.n_det, self.n_freq, stream)

    def heterodyne_setup(self, theta0, n_bins: int, bin_rule: int = 0):
        return heterodyne_setup(self._ctx, theta0, n_bins, bin_rule)

    def loglike_uneven(self, theta, subs, marg=GW_MARG_NONE, prec=GW_PREC_FP64, use_graph=True, out=None,
                       stream=None):
        return loglike_batch_uneven(self._ctx, theta, subs, GW_HET, marg, prec, use_graph, out, stream)

    def set_het_shape(self, waves_per_block: int = 4, grid: int = 0, n_ech: int = 0):
        gw_set_het_shape(self._ctx, waves_per_block, grid, n_ech)

    def data_inner(self) -> float:
        return gw_data_inner(self._ctx)

    def set_full_kernel(self, kind: int = 0):
        """0 automatic, 1 vector-ALU reduction, 2 matrix-core reduction (mixed precision)."""
        gw_set_full_kernel(self._ctx, kind)

    @property
    def mom_blk(self) -> int:
        return gw_full_info(self._ctx)

    def set_full_shape(self, tpb: int = 0, n_chunks: int = 0):
        gw_set_full_shape(self._ctx, tpb, n_chunks)

    def close(self):
        if self._ctx is not None and self._ctx.value:
            gw_ctx_destroy(self._ctx)
        self._ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
