"""Constrained slice sampling and nested sampling, plain FP64 reference.

Sec. II.B (nested sampling, Eq. cprior): m live points; each iteration
deletes the k lowest-likelihood points, raises log L* to the largest deleted
log-likelihood (equivalent to k sequential deletions), accumulates their
volume contributions into the evidence and replaces them by constrained draws.
Sec. II.C / III.B (Eq. block_cprior): the constrained draw is a Gibbs sweep
over parameter blocks, each updated by a hit-and-run slice step along a random
direction drawn from the block covariance of the live points, with stepping
out and shrinking.

Readings used here (where the paper is silent):
* sampling space: the 11-dimensional unit cube of the synthetic prior
  [Mc, q, chi1, chi2, Lambda1, Lambda2, iota, ra, dec, psi, t_c], with d_L and
  phi_c marginalised;
* direction: u uniform on the unit sphere of the block (normalised Gaussian
  draws, Box-Muller from uniforms), d = L u with L the Cholesky factor of the
  block covariance; a block may hold every coordinate (the unblocked nested
  slice sampler of the sampler-configuration section, run with M d joint
  steps per iteration); bracket width w along t, placed at a uniform offset;
  stepping out with a budget of m = 2 max_out + 1 split at random between
  the two ends, J = floor(m V) steps for the lower end and m - 1 - J for the
  upper one (the stepping-out procedure of Neal 2003, Sec. 4.1, which keeps
  the move reversible when a cap binds); shrinking at most ``max_shrink``
  times, after which the chain keeps its point (status 1);
* a point outside the unit cube fails the constraint without an evaluation;
* random numbers: explicit uniforms per chain, laid out as
  [n_dir direction, 1 offset, 1 budget split V, max_shrink shrink draws] with
  n_dir = max(4, 2 ceil(b / 2)) for a block of b coordinates (one Box-Muller
  pair per two coordinates, at least two pairs); or Philox4x64-10
  (Salmon et al. 2011), uniform j of chain c from counter
  (counter_base, c, j // 4, 0) and key (seed, 0), output word j % 4,
  u = ((word >> 11) + 0.5) * 2^-53;
* evidence bookkeeping: the k deletions of an iteration are taken in order of
  increasing log L with live counts m, m-1, ..., m-k+1, ln X dropping by
  1/(live count) each; weight L_j (X_{j-1} - X_j); termination when
  ln(Z_dead + Z_live) - ln Z_dead < dlogz with Z_live = X mean(L_live); the
  final live points are added with equal shares of X.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import logsumexp

N_DIM = 11
PRIOR_LO = np.array([1.1, 0.5, -0.05, -0.05, 0.0, 0.0])
PRIOR_HI = np.array([1.4, 1.0, 0.05, 0.05, 5000.0, 5000.0])
BLOCKS = ((0, 1, 4, 5), (2,), (3,), (6,), (7, 8), (9,), (10,))
N_UNIFORM_FIXED = 6  # 4 direction + 1 offset + 1 budget split (blocks of up to 4 coordinates)

_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1


def prior_transform(u: np.ndarray) -> np.ndarray:
    """Unit-cube point [11] -> parameter vector [13] (d_L = 1, phi_c = 0)."""
    u = np.asarray(u, dtype=np.float64)
    th = np.zeros(13)
    th[:6] = PRIOR_LO + (PRIOR_HI - PRIOR_LO) * u[:6]
    th[6] = 1.0
    th[7] = math.acos(1.0 - 2.0 * u[6])
    th[8] = 2.0 * math.pi * u[7]
    th[9] = math.asin(2.0 * u[8] - 1.0)
    th[10] = math.pi * u[9]
    th[11] = 0.0
    th[12] = -0.1 + 0.2 * u[10]
    return th


def prior_transform_time(u: np.ndarray, d_lo: float, d_hi: float) -> np.ndarray:
    """Unit-cube point [11] -> parameter vector [13] when t_c is marginalised
    (the paper's GW170817 configuration samples d_L in its place): as
    ``prior_transform`` but coordinate 10 is d_L with a prior proportional to
    d_L^2 on [d_lo, d_hi] (inverse CDF d = (d_lo^3 + u (d_hi^3 - d_lo^3))^(1/3)),
    and t_c = 0 (ignored)."""
    th = prior_transform(u)
    lo3 = d_lo ** 3
    th[6] = (lo3 + float(u[10]) * (d_hi ** 3 - lo3)) ** (1.0 / 3.0)
    th[12] = 0.0
    return th


C_SI = 299792458.0  # m / s


def sky_frame_basis(det_pos: np.ndarray, a: int = 0, b: int = 1):
    """Unit baseline n = (r_b - r_a) / |r_b - r_a| of detectors a and b and an
    orthonormal pair across it: e1 is the Earth's axis z made orthogonal to n
    (x when n lies along z), e2 = n x e1."""
    base = np.asarray(det_pos[b], dtype=np.float64) - np.asarray(det_pos[a], dtype=np.float64)
    n = base / np.linalg.norm(base)
    ref = np.array([0.0, 0.0, 1.0])
    if abs(n @ ref) > 0.99:
        ref = np.array([1.0, 0.0, 0.0])
    e1 = ref - (ref @ n) * n
    e1 = e1 / np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    return n, e1, e2


def detector_frame_sky(u_az: float, u_zen: float, det_pos: np.ndarray, gmst: float = 0.0, a: int = 0,
                       b: int = 1):
    """(ra, dec) of the direction with azimuth 2 pi u_az and zenith
    acos(1 - 2 u_zen) about the baseline of detectors a and b (the detector
    sky frame of the blocked-kernel section); isotropic when u is uniform.
    Returns (ra, dec, s) with s the unit source direction (Earth-fixed)."""
    n, e1, e2 = sky_frame_basis(det_pos, a, b)
    kap = 2.0 * math.pi * u_az
    zen = math.acos(1.0 - 2.0 * u_zen)
    s = math.cos(zen) * n + math.sin(zen) * (math.cos(kap) * e1 + math.sin(kap) * e2)
    dec = math.asin(max(-1.0, min(1.0, float(s[2]))))
    ra = (math.atan2(float(s[1]), float(s[0])) + gmst) % (2.0 * math.pi)
    return ra, dec, s


def prior_transform_frame(u: np.ndarray, det_pos: np.ndarray, gmst: float = 0.0, a: int = 0, b: int = 1,
                          det_time: bool = False, d_range=None) -> np.ndarray:
    """``prior_transform`` (or ``prior_transform_time`` when d_range = (d_lo,
    d_hi)) with coordinates 7 and 8 read in the detector sky frame.  With
    det_time, coordinate 10 is the arrival time t_a at detector a, uniform on
    [-0.1, 0.1] s, and t_c = t_a + s . r_a / c (the detector-frame time that
    the same section suggests); the implied prior on the geocentre t_c is
    uniform only away from the ends of its range."""
    th = prior_transform(u) if d_range is None else prior_transform_time(u, *d_range)
    ra, dec, s = detector_frame_sky(float(u[7]), float(u[8]), det_pos, gmst, a, b)
    th[8], th[9] = ra, dec
    if det_time and d_range is None:
        th[12] = (-0.1 + 0.2 * float(u[10])) + float(s @ np.asarray(det_pos[a], dtype=np.float64)) / C_SI
    return th


def philox4x64(counter, key):
    """Philox4x64 with 10 rounds (Salmon, Moraes, Dror & Shaw 2011)."""
    c = [int(v) & _MASK for v in counter]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for _ in range(10):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> 64, p0 & _MASK
        hi1, lo1 = p1 >> 64, p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return c


def philox_uniforms(seed: int, counter_base: int, chain: int, n: int) -> np.ndarray:
    out = np.empty(n)
    block = None
    for j in range(n):
        if j % 4 == 0:
            block = philox4x64((counter_base, chain, j // 4, 0), (seed, 0))
        out[j] = ((block[j % 4] >> 11) + 0.5) * 2.0 ** -53
    return out


def n_direction_uniforms(b: int) -> int:
    """Uniforms spent on the direction of a block of b coordinates."""
    return max(4, 2 * ((b + 1) // 2))


def n_fixed_uniforms(b: int) -> int:
    """Uniforms before the shrink draws: direction, the bracket offset, then
    the split of the stepping-out budget."""
    return n_direction_uniforms(b) + 2


def direction(uni: np.ndarray, chol: np.ndarray) -> np.ndarray:
    """d = L u, u a unit vector from Box-Muller normals: pair p turns
    (uni[2p], uni[2p + 1]) into r cos(2 pi uni[2p + 1]), r sin(2 pi uni[2p + 1])
    with r = sqrt(-2 ln uni[2p]); the first b normals are used."""
    b = chol.shape[0]
    z = []
    for p in range(n_direction_uniforms(b) // 2):
        r = math.sqrt(-2.0 * math.log(uni[2 * p]))
        z += [r * math.cos(2 * math.pi * uni[2 * p + 1]), r * math.sin(2 * math.pi * uni[2 * p + 1])]
    z = np.array(z[:b])
    z = z / np.linalg.norm(z)
    return chol @ z


def slice_chain(x0, logl0, logl_star, block, chol, uni, loglike, w=1.0, max_out=10, max_shrink=100,
                screen=None, screen_margin=0.0, audit_frac=0.0, stats=None):
    """One hit-and-run slice update of one chain on one block.

    Returns (x, logl, n_evals, status, min_margin): status 1 when the shrink cap
    was hit (old point kept); min_margin = smallest |logL - logL*| seen, which
    tells a caller how close a comparison came to a tie.

    Learned prescreen (an addition; the paper's sampler evaluates every
    candidate): with ``screen`` a callable (x, kind, index) -> (prediction,
    audit uniform), for the index-th test of a kind (0 lower end, 1 upper
    end, 2 shrink draw, counted within the block), a candidate inside the
    cube gets its exact log L only when the prediction is at least
    log L* - screen_margin or the audit uniform is below audit_frac;
    otherwise it counts as outside the constraint with no evaluation.  The
    closest |prediction - cut| enters min_margin too.  ``stats`` (a dict)
    accumulates 'screened', 'audited' and 'audited_inside'.
    """
    x0 = np.asarray(x0, dtype=np.float64)
    idx = np.asarray(block)
    d = direction(uni, chol)
    n_evals = 0
    margin = math.inf

    def point(t):
        x = x0.copy()
        x[idx] = x0[idx] + t * d
        return x

    def ok(t, kind=0, index=0):
        nonlocal n_evals, margin
        x = point(t)
        if np.any(x[idx] < 0.0) or np.any(x[idx] > 1.0):
            return False, x, -math.inf
        audited = False
        if screen is not None:
            pred, u_audit = screen(x, kind, index)
            cut = logl_star - screen_margin
            margin = min(margin, abs(pred - cut))
            if not pred >= cut:
                if not u_audit < audit_frac:
                    if stats is not None:
                        stats["screened"] = stats.get("screened", 0) + 1
                    return False, x, -math.inf
                audited = True
        v = loglike(x)
        n_evals += 1
        margin = min(margin, abs(v - logl_star))
        if audited and stats is not None:
            stats["audited"] = stats.get("audited", 0) + 1
            stats["audited_inside"] = stats.get("audited_inside", 0) + int(v > logl_star)
        return v > logl_star, x, v

    nfix = n_fixed_uniforms(len(block))
    r = uni[nfix - 2]
    t_lo = -r * w
    t_hi = (1.0 - r) * w
    budget = 2 * max_out + 1
    j_lo = int(math.floor(budget * uni[nfix - 1]))
    j_hi = budget - 1 - j_lo
    for i in range(j_lo):
        good, _, _ = ok(t_lo, 0, i)
        if not good:
            break
        t_lo -= w
    for i in range(j_hi):
        good, _, _ = ok(t_hi, 1, i)
        if not good:
            break
        t_hi += w
    for s in range(max_shrink):
        t = t_lo + uni[nfix + s] * (t_hi - t_lo)
        good, x, v = ok(t, 2, s)
        if good:
            return x, v, n_evals, 0, margin
        if t < 0.0:
            t_lo = t
        else:
            t_hi = t
    return x0.copy(), logl0, n_evals, 1, margin


def block_cholesky(live: np.ndarray, block) -> np.ndarray:
    """Cholesky factor of the covariance of the live points on ``block``."""
    sub = np.asarray(live)[:, list(block)]
    cov = np.atleast_2d(np.cov(sub, rowvar=False))
    cov = cov + 1e-12 * np.eye(cov.shape[0])
    return np.linalg.cholesky(cov)


def nested_sampling(loglike, n_live: int, n_delete: int, seed: int, dlogz: float = 0.1, blocks=BLOCKS,
                    n_dim: int = N_DIM, max_iter: int = 100000, sweeps: int = 1, w: float = 1.0,
                    max_out: int = 10, max_shrink: int = 100):
    """Slice-within-Gibbs nested sampling; returns a dict with logZ, H, counts."""
    rng = np.random.default_rng(seed)
    live = rng.uniform(size=(n_live, n_dim))
    logl = np.array([loglike(x) for x in live])
    n_evals = n_live
    dead_logl, dead_logw = [], []
    log_x = 0.0
    it = 0
    counter = 0
    while it < max_iter:
        order = np.argsort(logl, kind="stable")
        worst = order[:n_delete]
        logl_star = float(logl[worst[-1]])
        for j, i in enumerate(worst):
            new_log_x = log_x - 1.0 / (n_live - j)
            dead_logl.append(float(logl[i]))
            dead_logw.append(float(logl[i]) + log_x + math.log1p(-math.exp(new_log_x - log_x)))
            log_x = new_log_x
        survivors = order[n_delete:]
        starts = rng.choice(survivors, size=n_delete, replace=True)
        chols = [block_cholesky(live[survivors], b) for b in blocks]
        new_x = live[starts].copy()
        new_l = logl[starts].copy()
        for _ in range(sweeps):
            for bi, b in enumerate(blocks):
                for c in range(n_delete):
                    uni = philox_uniforms(seed, counter, c, n_fixed_uniforms(len(b)) + max_shrink)
                    x, v, ne, st, _ = slice_chain(new_x[c], new_l[c], logl_star, b, chols[bi], uni, loglike,
                                                  w, max_out, max_shrink)
                    new_x[c], new_l[c] = x, v
                    n_evals += ne
                counter += 1
        live[worst] = new_x
        logl[worst] = new_l
        it += 1
        log_z_dead = logsumexp(dead_logw)
        log_z_live = log_x + logsumexp(logl) - math.log(n_live)
        if np.logaddexp(log_z_dead, log_z_live) - log_z_dead < dlogz:
            break
    all_logw = np.concatenate([dead_logw, logl + log_x - math.log(n_live)])
    all_logl = np.concatenate([dead_logl, logl])
    log_z = float(logsumexp(all_logw))
    p = np.exp(all_logw - log_z)
    h = float(np.sum(p * all_logl) - log_z)
    return dict(log_z=log_z, h=h, log_z_err=math.sqrt(max(h, 0.0) / n_live), iterations=it, n_evals=n_evals,
                live=live, logl=logl, dead_logl=np.array(dead_logl), dead_logw=np.array(dead_logw))
