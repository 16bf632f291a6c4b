"""ctypes binding of libgwswig.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/gwswig.h with
the same name; all arithmetic happens in the library's HIP kernels.  Device
buffers are torch CUDA tensors (PyTorch provides device memory and streams).
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgwswig.so")

GW_OK, GW_EINVAL, GW_ENOMEM, GW_EDEVICE, GW_ESTATE, GW_ENOTSUP = 0, -1, -2, -3, -4, -5
GW_FULL, GW_HET = 0, 1
GW_MARG_NONE, GW_MARG_PHASE, GW_MARG_PHASE_DIST, GW_MARG_PHASE_TIME = 0, 1, 2, 3
GW_PREC_FP64, GW_PREC_MIXED = 0, 1
GW_MAX_DET = 4
GW_NPARAM = 13
GW_MAX_BLOCK = 11  # coordinates per slice block (a block may hold all 11)

_STATUS_NAMES = {0: "GW_OK", -1: "GW_EINVAL", -2: "GW_ENOMEM", -3: "GW_EDEVICE", -4: "GW_ESTATE", -5: "GW_ENOTSUP"}


class GwError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class gw_problem(ctypes.Structure):
    _fields_ = [
        ("n_det", ctypes.c_int32),
        ("k0", ctypes.c_int64),
        ("n_freq", ctypes.c_int64),
        ("df", ctypes.c_double),
        ("data_re", ctypes.POINTER(ctypes.c_double)),
        ("data_im", ctypes.POINTER(ctypes.c_double)),
        ("psd", ctypes.POINTER(ctypes.c_double)),
        ("det_tensor", ctypes.POINTER(ctypes.c_double)),
        ("det_pos", ctypes.POINTER(ctypes.c_double)),
        ("gmst", ctypes.c_double),
        ("dist_grid", ctypes.POINTER(ctypes.c_double)),
        ("dist_logw", ctypes.POINTER(ctypes.c_double)),
        ("n_dist", ctypes.c_int32),
    ]


class gw_slice_args(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int64),
        ("x", ctypes.c_void_p),
        ("logl", ctypes.c_void_p),
        ("logl_star", ctypes.c_double),
        ("block", ctypes.POINTER(ctypes.c_int32)),
        ("block_dim", ctypes.c_int32),
        ("chol", ctypes.POINTER(ctypes.c_double)),
        ("seed", ctypes.c_uint64),
        ("counter", ctypes.c_uint64),
        ("uniforms", ctypes.c_void_p),
        ("w", ctypes.c_double),
        ("max_out", ctypes.c_int32),
        ("max_shrink", ctypes.c_int32),
        ("like", ctypes.c_int32),
        ("marg", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("n_evals", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("use_graph", ctypes.c_int32),
        ("mlp", ctypes.c_void_p),
        ("margin", ctypes.c_double),
        ("audit_frac", ctypes.c_double),
        ("screen_stats", ctypes.POINTER(ctypes.c_int64)),
        ("rec_x", ctypes.c_void_p),
        ("rec_logl", ctypes.c_void_p),
        ("rec_cap", ctypes.c_int64),
        ("rec_count", ctypes.c_void_p),
    ]


class gw_sweep_args(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int64),
        ("x", ctypes.c_void_p),
        ("logl", ctypes.c_void_p),
        ("logl_star", ctypes.c_double),
        ("n_blocks", ctypes.c_int32),
        ("block_dim", ctypes.POINTER(ctypes.c_int32)),
        ("block", ctypes.POINTER(ctypes.c_int32)),
        ("chol", ctypes.POINTER(ctypes.c_double)),
        ("seed", ctypes.c_uint64),
        ("counter", ctypes.c_uint64),
        ("w", ctypes.c_double),
        ("max_out", ctypes.c_int32),
        ("max_shrink", ctypes.c_int32),
        ("like", ctypes.c_int32),
        ("marg", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("n_evals", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("use_graph", ctypes.c_int32),
        ("use_cache", ctypes.c_int32),
        ("eval_kinds", ctypes.POINTER(ctypes.c_int64)),
        ("mlp", ctypes.c_void_p),
        ("margin", ctypes.c_double),
        ("audit_frac", ctypes.c_double),
        ("screen_stats", ctypes.POINTER(ctypes.c_int64)),
        ("rec_x", ctypes.c_void_p),
        ("rec_logl", ctypes.c_void_p),
        ("rec_cap", ctypes.c_int64),
        ("rec_count", ctypes.c_void_p),
    ]


class gw_fiducial_args(ctypes.Structure):
    _fields_ = [
        ("pop", ctypes.c_int64),
        ("generations", ctypes.c_int32),
        ("f_scale", ctypes.c_double),
        ("cr", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("lo", ctypes.POINTER(ctypes.c_double)),
        ("hi", ctypes.POINTER(ctypes.c_double)),
        ("prec", ctypes.c_int32),
    ]


_LIB = None

_P = ctypes.c_void_p
_SIGS = {
    "gw_last_error": (ctypes.c_char_p, []),
    "gw_version": (ctypes.c_char_p, []),
    "gw_ctx_create": (ctypes.c_int, [ctypes.POINTER(gw_problem), ctypes.c_int32, ctypes.POINTER(_P)]),
    "gw_ctx_destroy": (ctypes.c_int, [_P]),
    "gw_data_inner": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "loglike_batch": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "loglike_batch_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "gw_template": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
    "gw_set_full_shape": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "gw_profile_enable": (ctypes.c_int, [_P, ctypes.c_int32]),
    "heterodyne_setup": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_double)]),
    "gw_het_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "loglike_batch_uneven": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "gw_set_het_shape": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "gw_set_het_tm_split": (ctypes.c_int, [_P, ctypes.c_int32]),
    "gw_autotune": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                   _P]),
    "gw_graph_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "slice_step": (ctypes.c_int, [_P, ctypes.POINTER(gw_slice_args), _P]),
    "slice_sweep": (ctypes.c_int, [_P, ctypes.POINTER(gw_sweep_args), _P]),
    "gw_set_time_window": (ctypes.c_int, [_P, ctypes.c_double]),
    "gw_set_time_oversample": (ctypes.c_int, [_P, ctypes.c_int32]),
    "gw_time_grid_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "gw_wcache_create": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(_P)]),
    "gw_wcache_destroy": (ctypes.c_int, [_P]),
    "gw_wcache_update": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "gw_wcache_loglike": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         _P, _P]),
    "gw_prior_transform": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
    "gw_prior_transform_marg": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, _P, _P]),
    "gw_set_full_kernel": (ctypes.c_int, [_P, ctypes.c_int32]),
    "gw_full_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "gw_full_phase_runs": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "gw_phasor_gain": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "gw_mlp_create": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "gw_mlp_destroy": (ctypes.c_int, [_P]),
    "gw_mlp_n_params": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64)]),
    "gw_mlp_set_scaling": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                          ctypes.c_double, ctypes.c_double]),
    "gw_mlp_set_params": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float)]),
    "gw_mlp_get_params": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float)]),
    "gw_mlp_grad": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_float),
                                   ctypes.POINTER(ctypes.c_float), _P]),
    "gw_mlp_train_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.c_float, ctypes.POINTER(ctypes.c_float),
                                         _P]),
    "gw_mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int32, _P]),
    "gw_prescreen_batch": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, _P, _P, _P, ctypes.POINTER(ctypes.c_int64), _P]),
    "gw_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "gw_fiducial_search": (ctypes.c_int, [_P, ctypes.POINTER(gw_fiducial_args), _P, _P,
                                          ctypes.POINTER(ctypes.c_double), _P]),
    "gw_set_sky_frame": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "gw_reconstruct": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                                      ctypes.c_int32, _P, _P, _P, _P]),
}


def load(path: str = LIB_PATH):
    """Load the library once; raise if it is missing (no fallback exists)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2607_28265_amd.build` "
                           "(there is no CPU fallback)")
    # Device memory and streams come from torch, which brings its own HIP
    # runtime: start it before the library is loaded, so that the library
    # binds to the runtime already in the process instead of starting a
    # second one (a second runtime started first leaves torch without GPUs).
    try:
        import torch
        torch.cuda.is_available()
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def register(name: str, restype, argtypes):
    """Declare an additional exported symbol's signature."""
    _SIGS[name] = (restype, argtypes)
    if _LIB is not None:
        fn = getattr(_LIB, name)
        fn.restype = restype
        fn.argtypes = argtypes


def gw_last_error() -> str:
    return load().gw_last_error().decode()


def gw_version() -> str:
    return load().gw_version().decode()


def check(status: int, where: str):
    if status != GW_OK:
        raise GwError(status, where, gw_last_error())


def _dptr(arr):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _tensor_ptr(t):
    return ctypes.c_void_p(int(t.data_ptr()))


def gw_ctx_create(prob, device: int = 0) -> ctypes.c_void_p:
    """Create a context from a problem object (see gwsynth.Problem)."""
    import numpy as np
    lib = load()
    data = np.ascontiguousarray(prob.data)
    keep = dict(
        re=np.ascontiguousarray(data.real, dtype=np.float64),
        im=np.ascontiguousarray(data.imag, dtype=np.float64),
        psd=np.ascontiguousarray(prob.psd, dtype=np.float64),
        ten=np.ascontiguousarray(prob.det_tensor, dtype=np.float64),
        pos=np.ascontiguousarray(prob.det_pos, dtype=np.float64),
        dg=np.ascontiguousarray(prob.dist_grid, dtype=np.float64),
        dw=np.ascontiguousarray(prob.dist_logw, dtype=np.float64),
    )
    p = gw_problem(n_det=data.shape[0], k0=int(prob.k0), n_freq=int(prob.n_freq), df=float(prob.df),
                   data_re=_dptr(keep["re"]), data_im=_dptr(keep["im"]), psd=_dptr(keep["psd"]),
                   det_tensor=_dptr(keep["ten"]), det_pos=_dptr(keep["pos"]), gmst=float(prob.gmst),
                   dist_grid=_dptr(keep["dg"]), dist_logw=_dptr(keep["dw"]), n_dist=len(keep["dg"]))
    out = ctypes.c_void_p()
    check(lib.gw_ctx_create(ctypes.byref(p), device, ctypes.byref(out)), "gw_ctx_create")
    return out


def gw_ctx_destroy(ctx):
    check(load().gw_ctx_destroy(ctx), "gw_ctx_destroy")


def gw_data_inner(ctx) -> float:
    v = ctypes.c_double()
    check(load().gw_data_inner(ctx, ctypes.byref(v)), "gw_data_inner")
    return v.value


def _check_theta(theta):
    import torch
    if not (theta.is_cuda and theta.dtype == torch.float64 and theta.dim() == 2 and theta.shape[1] == GW_NPARAM
            and theta.is_contiguous()):
        raise ValueError("theta must be a contiguous CUDA float64 tensor of shape [n, 13]")


def loglike_batch(ctx, theta, like: int = GW_FULL, marg: int = GW_MARG_NONE, prec: int = GW_PREC_FP64,
                  out=None, stream=None):
    """log L for every row of ``theta`` (CUDA float64 [n, 13]) -> CUDA float64 [n]."""
    import torch
    _check_theta(theta)
    n = theta.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=theta.device)
    elif not (out.is_cuda and out.dtype == torch.float64 and out.numel() >= n and out.is_contiguous()):
        raise ValueError("out must be a contiguous CUDA float64 tensor with at least n elements")
    check(load().loglike_batch(ctx, _tensor_ptr(theta), n, like, marg, prec, _tensor_ptr(out), _stream_ptr(stream)),
          "loglike_batch")
    return out


GW_NOALLOC_DOUBLES = 1 << 21


def noalloc_max_rows(n_det: int) -> int:
    """Largest batch of loglike_batch_noalloc for ``n_det`` detectors."""
    return GW_NOALLOC_DOUBLES // (34 + 16 * n_det)


def loglike_batch_noalloc(ctx, theta, marg: int = GW_MARG_NONE, prec: int = GW_PREC_FP64, out=None, stream=None):
    """Allocation-free full-band log-likelihood of theta [n, 13] (CUDA float64)."""
    import torch
    _check_theta(theta)
    n = theta.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=theta.device)
    check(load().loglike_batch_noalloc(ctx, _tensor_ptr(theta), n, int(marg), int(prec), _tensor_ptr(out),
                                       _stream_ptr(stream)), "loglike_batch_noalloc")
    return out


def gw_template(ctx, theta, n_det: int, n_freq: int, stream=None):
    """Projected templates -> CUDA complex128 [n, n_det, n_freq]."""
    import torch
    _check_theta(theta)
    n = theta.shape[0]
    h = torch.empty((n, n_det, n_freq, 2), dtype=torch.float64, device=theta.device)
    check(load().gw_template(ctx, _tensor_ptr(theta), n, _tensor_ptr(h), _stream_ptr(stream)), "gw_template")
    return torch.view_as_complex(h)


def gw_set_full_shape(ctx, tpb: int, n_chunks: int):
    check(load().gw_set_full_shape(ctx, tpb, n_chunks), "gw_set_full_shape")


def gw_set_full_kernel(ctx, kind: int):
    check(load().gw_set_full_kernel(ctx, kind), "gw_set_full_kernel")


def gw_full_phase_runs(ctx):
    """(k_min, len): the run levels of the mixed reduction's phase recurrence."""
    k = (ctypes.c_int32 * 4)()
    n = (ctypes.c_int32 * 4)()
    check(load().gw_full_phase_runs(ctx, k, n), "gw_full_phase_runs")
    return list(k), list(n)


def gw_full_info(ctx) -> int:
    v = ctypes.c_int32()
    check(load().gw_full_info(ctx, ctypes.byref(v)), "gw_full_info")
    return v.value


def gw_phasor_gain(ctx):
    re, im = ctypes.c_double(), ctypes.c_double()
    check(load().gw_phasor_gain(ctx, ctypes.byref(re), ctypes.byref(im)), "gw_phasor_gain")
    return complex(re.value, im.value)


def gw_profile_enable(ctx, enable=True):
    """enable: True/1 the dominant kernel, 2 the time-grid kernel, False/0 off."""
    check(load().gw_profile_enable(ctx, int(enable)), "gw_profile_enable")


def gw_profile_read(ctx):
    """(summed kernel ms, number of timed launches) since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    check(load().gw_profile_read(ctx, ctypes.byref(ms), ctypes.byref(n)), "gw_profile_read")
    return ms.value, n.value


def heterodyne_setup(ctx, theta0, n_bins: int, bin_rule: int = 0):
    """Build the relative-binning summary data; returns the edge frequencies (numpy)."""
    import numpy as np
    th = np.ascontiguousarray(theta0, dtype=np.float64)
    if th.shape != (GW_NPARAM,):
        raise ValueError("theta0 must have 13 entries")
    edges = np.zeros(n_bins + 1)
    check(load().heterodyne_setup(ctx, _dptr(th), n_bins, bin_rule, _dptr(edges)), "heterodyne_setup")
    nb = gw_het_info(ctx)
    return edges[:nb + 1]


def gw_het_info(ctx) -> int:
    v = ctypes.c_int32()
    check(load().gw_het_info(ctx, ctypes.byref(v)), "gw_het_info")
    return v.value


def loglike_batch_uneven(ctx, theta, subs, like: int = GW_HET, marg: int = GW_MARG_NONE,
                         prec: int = GW_PREC_FP64, use_graph: bool = True, out=None, stream=None):
    """Sub-batches ``subs`` (CUDA int64 [n_sub, 2] of (row offset, count)) in one launch sequence."""
    import torch
    _check_theta(theta)
    if not (subs.is_cuda and subs.dtype == torch.int64 and subs.is_contiguous() and subs.dim() == 2
            and subs.shape[1] == 2):
        raise ValueError("subs must be a contiguous CUDA int64 tensor of shape [n_sub, 2]")
    n = theta.shape[0]
    if out is None:
        out = torch.full((n,), float("nan"), dtype=torch.float64, device=theta.device)
    check(load().loglike_batch_uneven(ctx, _tensor_ptr(theta), n, _tensor_ptr(subs), subs.shape[0], like, marg,
                                      prec, 1 if use_graph else 0, _tensor_ptr(out), _stream_ptr(stream)),
          "loglike_batch_uneven")
    return out


def gw_set_het_shape(ctx, waves_per_block: int, grid: int, n_ech: int = 0):
    check(load().gw_set_het_shape(ctx, waves_per_block, grid, n_ech), "gw_set_het_shape")


def gw_graph_info(ctx):
    n = ctypes.c_int32()
    ms = ctypes.c_double()
    check(load().gw_graph_info(ctx, ctypes.byref(n), ctypes.byref(ms)), "gw_graph_info")
    return n.value, ms.value


def gw_autotune(ctx, theta, like: int, marg: int, prec: int, reps: int = 3, stream=None):
    """Pick the fastest launch shape on ``theta``; returns ((a, b, c), ms per call)."""
    _check_theta(theta)
    shape = (ctypes.c_int32 * 3)()
    ms = ctypes.c_double()
    check(load().gw_autotune(ctx, _tensor_ptr(theta), theta.shape[0], like, marg, prec, reps, shape,
                             ctypes.byref(ms), _stream_ptr(stream)), "gw_autotune")
    return (shape[0], shape[1], shape[2]), ms.value


def slice_uniforms_fixed(block_dim: int) -> int:
    """Uniforms of a slice update before its shrink draws (GW_SLICE_UNI_FIXED)."""
    return (4 if block_dim <= 4 else 2 * ((block_dim + 1) // 2)) + 2


def _set_screen(a, prescreen, screen_stats):
    """Prescreen fields of a slice/sweep argument block: ``prescreen`` is None
    or (Mlp, margin, audit_frac); ``screen_stats`` a dict that receives the
    counts (screened out, audited, audited and inside)."""
    buf = (ctypes.c_int64 * 3)()
    if prescreen is not None:
        net, margin, audit = prescreen
        a.mlp = net._m.value if isinstance(net._m, ctypes.c_void_p) else net._m
        a.margin = float(margin)
        a.audit_frac = float(audit)
        if screen_stats is not None:
            a.screen_stats = buf
    return buf


def _set_record(a, record):
    """``record`` = (x [cap, 11], logl [cap], count [1] int64) CUDA tensors or None."""
    if record is None:
        return
    import torch
    rx, rl, rc = record
    if not (rx.is_cuda and rx.dtype == torch.float64 and rx.is_contiguous() and rx.dim() == 2 and rx.shape[1] == 11
            and rl.is_cuda and rl.dtype == torch.float64 and rl.numel() == rx.shape[0]
            and rc.is_cuda and rc.dtype == torch.int64 and rc.numel() == 1):
        raise ValueError("record = (x [cap, 11] float64, logl [cap] float64, count [1] int64), CUDA tensors")
    a.rec_x, a.rec_logl, a.rec_cap, a.rec_count = rx.data_ptr(), rl.data_ptr(), rx.shape[0], rc.data_ptr()


def _fill_screen(buf, prescreen, screen_stats):
    if prescreen is not None and screen_stats is not None:
        screen_stats.update(screened=int(buf[0]), audited=int(buf[1]), audited_inside=int(buf[2]))


def slice_step(ctx, x, logl, logl_star: float, block, chol, seed: int = 0, counter: int = 0, uniforms=None,
               w: float = 1.0, max_out: int = 10, max_shrink: int = 100, like: int = GW_HET,
               marg: int = GW_MARG_PHASE_DIST, prec: int = GW_PREC_FP64, n_evals=None, status=None, stream=None,
               use_graph: bool = True, prescreen=None, screen_stats=None, record=None):
    """One slice update of one block for every chain; x [k, 11] and logl [k] (CUDA float64) change in place.
    ``prescreen`` = (Mlp, margin, audit_frac) screens candidates with the network; ``record`` = (x, logl,
    count) CUDA tensors collect every exactly evaluated candidate (see gwswig.h)."""
    import numpy as np
    import torch
    if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous() and x.dim() == 2 and x.shape[1] == 11):
        raise ValueError("x must be a contiguous CUDA float64 tensor of shape [k, 11]")
    k = x.shape[0]
    if not (logl.is_cuda and logl.dtype == torch.float64 and logl.is_contiguous() and logl.numel() == k):
        raise ValueError("logl must be a contiguous CUDA float64 tensor with k entries")
    blk = np.ascontiguousarray(block, dtype=np.int32)
    ch = np.ascontiguousarray(chol, dtype=np.float64).reshape(len(blk), len(blk))
    nfix = slice_uniforms_fixed(len(blk))
    if uniforms is not None and not (uniforms.is_cuda and uniforms.dtype == torch.float64
                                     and uniforms.is_contiguous() and uniforms.shape == (k, nfix + max_shrink)):
        raise ValueError(f"uniforms must be a contiguous CUDA float64 tensor of shape [k, {nfix} + max_shrink]")
    for t in (n_evals, status):
        if t is not None and not (t.is_cuda and t.dtype == torch.int32 and t.numel() == k and t.is_contiguous()):
            raise ValueError("n_evals / status must be contiguous CUDA int32 tensors with k entries")
    a = gw_slice_args(k=k, x=x.data_ptr(), logl=logl.data_ptr(), logl_star=float(logl_star),
                      block=blk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), block_dim=len(blk),
                      chol=ch.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), seed=int(seed), counter=int(counter),
                      uniforms=uniforms.data_ptr() if uniforms is not None else None, w=float(w),
                      max_out=int(max_out), max_shrink=int(max_shrink), like=int(like), marg=int(marg),
                      prec=int(prec), n_evals=n_evals.data_ptr() if n_evals is not None else None,
                      status=status.data_ptr() if status is not None else None, use_graph=1 if use_graph else 0)
    buf = _set_screen(a, prescreen, screen_stats)
    _set_record(a, record)
    check(load().slice_step(ctx, ctypes.byref(a), _stream_ptr(stream)), "slice_step")
    _fill_screen(buf, prescreen, screen_stats)


def _check_chains(x, logl, n_evals, status):
    import torch
    if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous() and x.dim() == 2 and x.shape[1] == 11):
        raise ValueError("x must be a contiguous CUDA float64 tensor of shape [k, 11]")
    k = x.shape[0]
    if not (logl.is_cuda and logl.dtype == torch.float64 and logl.is_contiguous() and logl.numel() == k):
        raise ValueError("logl must be a contiguous CUDA float64 tensor with k entries")
    for t in (n_evals, status):
        if t is not None and not (t.is_cuda and t.dtype == torch.int32 and t.numel() == k and t.is_contiguous()):
            raise ValueError("n_evals / status must be contiguous CUDA int32 tensors with k entries")
    return k


def slice_sweep(ctx, x, logl, logl_star: float, blocks, chols, seed: int = 0, counter: int = 0, w: float = 1.0,
                max_out: int = 10, max_shrink: int = 100, like: int = GW_HET, marg: int = GW_MARG_PHASE_DIST,
                prec: int = GW_PREC_FP64, n_evals=None, status=None, stream=None, use_graph: bool = True,
                use_cache: bool = False, prescreen=None, screen_stats=None, record=None):
    """One sweep over ``blocks`` (list of index lists, with their Cholesky
    factors ``chols``) for every chain, block b with Philox counter
    counter + b; x [k, 11] and logl [k] change in place.  Returns the
    evaluations by kind (full, cached waveform, cached sums) with the
    waveform cache, else None.  ``prescreen`` / ``screen_stats`` as for
    slice_step."""
    import numpy as np
    k = _check_chains(x, logl, n_evals, status)
    nb = len(blocks)
    if not 1 <= nb <= 16 or len(chols) != nb:
        raise ValueError("1..16 blocks, one Cholesky factor each")
    bd = np.zeros(nb, np.int32)
    blk = np.zeros((nb, GW_MAX_BLOCK), np.int32)
    ch = np.zeros((nb, GW_MAX_BLOCK, GW_MAX_BLOCK), np.float64)
    for b, (idx, L) in enumerate(zip(blocks, chols)):
        idx = np.asarray(idx, dtype=np.int32).ravel()
        if not 1 <= idx.size <= GW_MAX_BLOCK:
            raise ValueError(f"each block has 1..{GW_MAX_BLOCK} coordinates")
        bd[b] = idx.size
        blk[b, :idx.size] = idx
        ch[b, :idx.size, :idx.size] = np.asarray(L, dtype=np.float64).reshape(idx.size, idx.size)
    a = gw_sweep_args(k=k, x=x.data_ptr(), logl=logl.data_ptr(), logl_star=float(logl_star), n_blocks=nb,
                      block_dim=bd.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                      block=blk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                      chol=ch.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), seed=int(seed), counter=int(counter),
                      w=float(w), max_out=int(max_out), max_shrink=int(max_shrink), like=int(like), marg=int(marg),
                      prec=int(prec), n_evals=n_evals.data_ptr() if n_evals is not None else None,
                      status=status.data_ptr() if status is not None else None, use_graph=1 if use_graph else 0,
                      use_cache=1 if use_cache else 0)
    kinds = (ctypes.c_int64 * 3)()
    if use_cache:
        a.eval_kinds = kinds
    buf = _set_screen(a, prescreen, screen_stats)
    _set_record(a, record)
    check(load().slice_sweep(ctx, ctypes.byref(a), _stream_ptr(stream)), "slice_sweep")
    _fill_screen(buf, prescreen, screen_stats)
    return (kinds[0], kinds[1], kinds[2]) if use_cache else None


def gw_prior_transform(ctx, x, stream=None, marg: int = GW_MARG_PHASE_DIST):
    """Unit-cube points (CUDA float64 [n, 11]) -> parameter vectors [n, 13]
    (coordinate 10 is t_c, or d_L with marg = GW_MARG_PHASE_TIME)."""
    import torch
    if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous() and x.dim() == 2 and x.shape[1] == 11):
        raise ValueError("x must be a contiguous CUDA float64 tensor of shape [n, 11]")
    th = torch.empty((x.shape[0], GW_NPARAM), dtype=torch.float64, device=x.device)
    check(load().gw_prior_transform_marg(ctx, _tensor_ptr(x), x.shape[0], int(marg), _tensor_ptr(th),
                                         _stream_ptr(stream)), "gw_prior_transform")
    return th


def _fptr(arr):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _check_unit(x):
    import torch
    if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous() and x.dim() == 2 and x.shape[1] == 11):
        raise ValueError("x must be a contiguous CUDA float64 tensor of shape [n, 11]")


class Mlp:
    """Owns one prescreen network on the context's device."""

    def __init__(self, ctx, seed: int = 7):
        self.ctx = ctx
        self._m = ctypes.c_void_p()
        check(load().gw_mlp_create(ctx.handle, seed, ctypes.byref(self._m)), "gw_mlp_create")

    @staticmethod
    def n_params() -> int:
        v = ctypes.c_int64()
        check(load().gw_mlp_n_params(ctypes.byref(v)), "gw_mlp_n_params")
        return v.value

    def set_scaling(self, x_mean, x_std, y_mean: float, y_std: float):
        import numpy as np
        xm = np.ascontiguousarray(x_mean, dtype=np.float64)
        xs = np.ascontiguousarray(x_std, dtype=np.float64)
        check(load().gw_mlp_set_scaling(self._m, _dptr(xm), _dptr(xs), float(y_mean), float(y_std)),
              "gw_mlp_set_scaling")

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        check(load().gw_mlp_set_params(self._m, _fptr(p)), "gw_mlp_set_params")

    def get_params(self):
        import numpy as np
        p = np.empty(self.n_params(), dtype=np.float32)
        check(load().gw_mlp_get_params(self._m, _fptr(p)), "gw_mlp_get_params")
        return p

    def grad(self, x, logl, stream=None):
        import numpy as np
        _check_unit(x)
        g = np.empty(self.n_params(), dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        check(load().gw_mlp_grad(self._m, _tensor_ptr(x), _tensor_ptr(logl), x.shape[0], _fptr(g), _fptr(loss),
                                 _stream_ptr(stream)), "gw_mlp_grad")
        return g, float(loss[0])

    def train_step(self, x, logl, lr: float, want_loss: bool = False, stream=None):
        import numpy as np
        _check_unit(x)
        loss = np.zeros(1, dtype=np.float32)
        check(load().gw_mlp_train_step(self._m, _tensor_ptr(x), _tensor_ptr(logl), x.shape[0], float(lr),
                                       _fptr(loss) if want_loss else None, _stream_ptr(stream)), "gw_mlp_train_step")
        return float(loss[0]) if want_loss else None

    def forward(self, x, bf16: bool = True, out=None, stream=None):
        import torch
        _check_unit(x)
        if out is None:
            out = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
        check(load().gw_mlp_forward(self._m, _tensor_ptr(x), x.shape[0], _tensor_ptr(out), 1 if bf16 else 0,
                                    _stream_ptr(stream)), "gw_mlp_forward")
        return out

    def prescreen(self, x, logl_star: float, margin: float, audit_frac: float = 0.01, seed: int = 7,
                  use_mlp: bool = True, like: int = GW_FULL, prec: int = GW_PREC_MIXED, stream=None):
        """(exact log L or -inf, flags, predictions, number of exact evaluations)."""
        import torch
        _check_unit(x)
        n = x.shape[0]
        logl = torch.empty(n, dtype=torch.float64, device=x.device)
        pred = torch.empty(n, dtype=torch.float64, device=x.device)
        flags = torch.empty(n, dtype=torch.int32, device=x.device)
        ne = ctypes.c_int64()
        check(load().gw_prescreen_batch(self.ctx.handle, self._m, _tensor_ptr(x), n, float(logl_star), float(margin),
                                        float(audit_frac), int(seed), 1 if use_mlp else 0, like, prec,
                                        _tensor_ptr(logl), _tensor_ptr(pred), _tensor_ptr(flags), ctypes.byref(ne),
                                        _stream_ptr(stream)), "gw_prescreen_batch")
        return logl, flags, pred, ne.value

    def close(self):
        if self._m is not None and self._m.value:
            load().gw_mlp_destroy(self._m)
        self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WaveformCache:
    """Slow / fast likelihood pair over ``n_slots`` cached waveforms (see
    gw_wcache_* in gwswig.h).  Slots are CUDA int32 tensors; parameter
    vectors CUDA float64 [n, 13]."""

    def __init__(self, ctx, n_slots: int):
        h = _P()
        check(load().gw_wcache_create(ctx, int(n_slots), ctypes.byref(h)), "gw_wcache_create")
        self._h = h
        self.n_slots = int(n_slots)

    def close(self):
        if self._h:
            load().gw_wcache_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _args(theta, slots, out):
        import torch
        _check_theta(theta)
        n = theta.shape[0]
        if not (slots.is_cuda and slots.dtype == torch.int32 and slots.is_contiguous() and slots.numel() == n):
            raise ValueError("slots must be a contiguous CUDA int32 tensor with one entry per row")
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=theta.device)
        elif not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= n):
            raise ValueError("out must be a contiguous CUDA float64 tensor with at least n elements")
        return n, out

    def update(self, theta, slots, marg: int = GW_MARG_PHASE_DIST, prec: int = GW_PREC_FP64, out=None, stream=None):
        n, out = self._args(theta, slots, out)
        check(load().gw_wcache_update(self._h, _tensor_ptr(theta), slots.data_ptr(), n, marg, prec, out.data_ptr(),
                                      _stream_ptr(stream)), "gw_wcache_update")
        return out

    def loglike(self, theta, slots, kind: int, marg: int = GW_MARG_PHASE_DIST, prec: int = GW_PREC_FP64, out=None,
                stream=None):
        n, out = self._args(theta, slots, out)
        check(load().gw_wcache_loglike(self._h, _tensor_ptr(theta), slots.data_ptr(), n, int(kind), marg, prec,
                                       out.data_ptr(), _stream_ptr(stream)), "gw_wcache_loglike")
        return out


def gw_set_time_window(ctx, window: float):
    """Half-width (s) of the uniform t_c prior of GW_MARG_PHASE_TIME."""
    check(load().gw_set_time_window(ctx, float(window)), "gw_set_time_window")


def gw_time_grid_info(ctx):
    """(delta, grid points, FFT length, bins per block) of the time marginal."""
    d = ctypes.c_double()
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(load().gw_time_grid_info(ctx, ctypes.byref(d), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
          "gw_time_grid_info")
    return d.value, a.value, b.value, c.value


def gw_reconstruct(ctx, theta, uniforms, like: int = GW_FULL, marg: int = GW_MARG_PHASE_DIST,
                   prec: int = GW_PREC_MIXED, n_phase: int = 2048, stream=None):
    """Post-hoc draws of (d_L, phi_c) for posterior samples ``theta``
    (CUDA float64 [n, 13]) with ``uniforms`` (CUDA float64 [n, 2]).  Returns
    (values [n, 2], grid indices int32 [n, 2], marginal log L [n])."""
    import torch
    if not (theta.is_cuda and theta.dtype == torch.float64 and theta.is_contiguous() and theta.dim() == 2
            and theta.shape[1] == GW_NPARAM):
        raise ValueError("theta must be a contiguous CUDA float64 tensor of shape [n, 13]")
    n = theta.shape[0]
    if not (uniforms.is_cuda and uniforms.dtype == torch.float64 and uniforms.is_contiguous()
            and tuple(uniforms.shape) == (n, 2)):
        raise ValueError("uniforms must be a contiguous CUDA float64 tensor of shape [n, 2]")
    out = torch.empty((n, 2), dtype=torch.float64, device=theta.device)
    idx = torch.empty((n, 2), dtype=torch.int32, device=theta.device)
    logl = torch.empty(n, dtype=torch.float64, device=theta.device)
    check(load().gw_reconstruct(ctx, _tensor_ptr(theta), n, int(like), int(marg), int(prec), _tensor_ptr(uniforms),
                                int(n_phase), _tensor_ptr(out), _tensor_ptr(idx), _tensor_ptr(logl),
                                _stream_ptr(stream)), "gw_reconstruct")
    return out, idx, logl


def gw_set_sky_frame(ctx, frame: int = 1, det_a: int = 0, det_b: int = 1, det_time: bool = False):
    """Sample the sky as zenith / azimuth about the baseline of detectors
    det_a -> det_b (frame 1) or as ra / dec (frame 0); det_time makes
    coordinate 10 the arrival time at det_a."""
    check(load().gw_set_sky_frame(ctx, int(frame), int(det_a), int(det_b), 1 if det_time else 0), "gw_set_sky_frame")


def gw_fiducial_search(ctx, x, generations: int, seed: int = 0, f_scale: float = 0.6, cr: float = 0.9, lo=None,
                       hi=None, prec: int = GW_PREC_MIXED, stream=None):
    """Differential-evolution search for the maximum of the full-band
    phase+distance marginal log L from population ``x`` (CUDA float64
    [pop, 11], updated in place).  Returns (log L of the final population
    [pop], best parameter vector [13] with d_L and phi_c at the peak)."""
    import numpy as np
    import torch
    if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous() and x.dim() == 2 and x.shape[1] == 11):
        raise ValueError("x must be a contiguous CUDA float64 tensor of shape [pop, 11]")
    fx = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
    lo_a = None if lo is None else np.ascontiguousarray(lo, dtype=np.float64).reshape(11)
    hi_a = None if hi is None else np.ascontiguousarray(hi, dtype=np.float64).reshape(11)
    a = gw_fiducial_args(pop=x.shape[0], generations=int(generations), f_scale=float(f_scale), cr=float(cr),
                         seed=int(seed), lo=_dptr(lo_a) if lo_a is not None else None,
                         hi=_dptr(hi_a) if hi_a is not None else None, prec=int(prec))
    best = np.zeros(13)
    check(load().gw_fiducial_search(ctx, ctypes.byref(a), _tensor_ptr(x), _tensor_ptr(fx), _dptr(best),
                                    _stream_ptr(stream)), "gw_fiducial_search")
    return fx, best


def gw_set_het_tm_split(ctx, n_chunks: int = 0):
    """Edge chunks of the heterodyned time marginal's edge moments (0 = heuristic)."""
    check(load().gw_set_het_tm_split(ctx, int(n_chunks)), "gw_set_het_tm_split")


def gw_set_time_oversample(ctx, factor: int = 4):
    """Grid points per sampling interval of the time marginal (1, 2, 4, 8, 16)."""
    check(load().gw_set_time_oversample(ctx, int(factor)), "gw_set_time_oversample")
