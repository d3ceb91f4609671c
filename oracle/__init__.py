"""CPU ORACLE — test infrastructure only.

Plain, slow CPU implementation of the TPC track-finding hot path (neighbour
links with FP32 decisions, mutual-link cleaning, cellular-automaton chains and
assignment, FP64 maximum-a-posteriori helix fit, FP64 Kalman diagnostic).
Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
import it; the GPU library never does, and it shares no code with the GPU path.

The arithmetic lives in ``tpcoracle.c`` (built with gcc, ``-ffp-contract=off``,
no fast-math). This module only marshals arguments. The rules it follows are
the readings of the paper adopted for this build (the paper, Sec. 1, names
the step -- CA seeding on pad-row links with time as the seeding coordinate
and a Kalman fit, derived from the Run 2 HLT tracker -- but gives no formulas):
see the header of ``tpcoracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "tpcoracle.c"), os.path.join(_HERE, "tpcmlp.c")]
_HDR = os.path.join(_HERE, "tpcoracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int32),
        ("row_x", ctypes.c_void_p),
        ("win_y", ctypes.c_float),
        ("win_t", ctypes.c_float),
        ("pair_c2", ctypes.c_float),
        ("max_gap", ctypes.c_int32),
        ("min_track_hits", ctypes.c_int32),
        ("bz", ctypes.c_double),
        ("sigma_y", ctypes.c_double),
        ("sigma_t", ctypes.c_double),
        ("ivar_s", ctypes.c_double),
        ("ivar_tau", ctypes.c_double),
        ("ivar_k", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("s_max", ctypes.c_double),
    ]


class _Fit(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("n_iter", ctypes.c_int32),
        ("ndf", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("x_ref", ctypes.c_double),
        ("y", ctypes.c_double),
        ("t", ctypes.c_double),
        ("sinphi", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("qpt", ctypes.c_double),
        ("chi2", ctypes.c_double),
        ("cov", ctypes.c_double * 15),
        ("init", ctypes.c_double * 5),
    ]


FIT_DTYPE = np.dtype([
    ("status", np.int32), ("n_iter", np.int32), ("ndf", np.int32), ("pad", np.int32),
    ("x_ref", np.float64), ("y", np.float64), ("t", np.float64), ("sinphi", np.float64),
    ("tau", np.float64), ("qpt", np.float64), ("chi2", np.float64),
    ("cov", np.float64, (15,)), ("init", np.float64, (5,)),
])


def build(force: bool = False) -> str:
    """Compile the oracle (plain C, gcc, no FP contraction, no fast-math)."""
    newest = max(os.path.getmtime(f) for f in _SRCS + [_HDR])
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                               "-mfpmath=sse", "-msse2", "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.ora_links.argtypes = [P, ctypes.c_int64, P, P, P, P, P, P]
        lib.ora_links_subset.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_int64, P, P, P, P]
        lib.ora_clean.argtypes = [ctypes.c_int64, P, P, P, P]
        lib.ora_tracks.argtypes = [P, ctypes.c_int64, P, P, P, P, P, P]
        lib.ora_tracks.restype = ctypes.c_int64
        lib.ora_chain_len.argtypes = [ctypes.c_int64, P, P, P]
        lib.ora_fit_map.argtypes = [P, ctypes.c_int32, P, P, P, P]
        lib.ora_fit_kf.argtypes = [P, ctypes.c_int32, P, P, P, ctypes.c_int32, P]
        lib.ora_fit_tracks.argtypes = [P, ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int32, P]
        lib.ora_map_cost.argtypes = [P, ctypes.c_int32, P, P, P, P, P]
        lib.ora_map_cost.restype = ctypes.c_double
        lib.ora_propagate_c.argtypes = [P, P, ctypes.c_double, P, P]
        lib.ora_propagate_c.restype = ctypes.c_int32
        lib.ora_sizeof_fit.restype = ctypes.c_int32
        lib.ora_sizeof_cfg.restype = ctypes.c_int32
        lib.ora_links_pruned.argtypes = [P, ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                         P, P, P, P]
        lib.ora_follow.argtypes = [P, P, ctypes.c_int64, P, P, P, ctypes.c_int64, P, P, P, P, P, P, P, P, P, P]
        lib.ora_follow.restype = ctypes.c_int64
        lib.ora_kf1_run.argtypes = [ctypes.c_int32, P, P, ctypes.c_float, ctypes.c_float, ctypes.c_float, P]
        lib.ora_kf1_run.restype = None
        lib.ora_triplets.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_int64, P, P]
        lib.ora_triplets.restype = ctypes.c_int64
        lib.ora_bf16.argtypes = [ctypes.c_float]
        lib.ora_bf16.restype = ctypes.c_float
        lib.ora_mlp_features.argtypes = [ctypes.c_float] * 9 + [ctypes.c_int32] + [ctypes.c_float] * 4 + \
            [ctypes.c_int32, P]
        lib.ora_mlp_forward_batch.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, P]
        lib.ora_mlp_grad.argtypes = [P, ctypes.c_int64, P, P, ctypes.c_double, ctypes.c_int32, P, P, P, P, P, P]
        lib.ora_mlp_grad.restype = ctypes.c_double
        lib.ora_mlp_sizeof.restype = ctypes.c_int32
        lib.ora_adamw_step.argtypes = [ctypes.c_int64, P, P, P, P, P] + [ctypes.c_double] * 5 + [ctypes.c_int32]
        assert lib.ora_mlp_sizeof() == 4 * MLP_NPARAM
        assert lib.ora_sizeof_fit() == ctypes.sizeof(_Fit) == FIT_DTYPE.itemsize
        assert lib.ora_sizeof_cfg() == ctypes.sizeof(_Cfg)
        _lib = lib
    return _lib


@dataclass
class Config:
    """Tracker constants (the readings of the paper adopted for this build)."""
    row_x: np.ndarray                 # float32[n_rows] pad-row x (cm)
    win_y: float = 1.5                # box half width in y per unit row gap (cm)
    win_t: float = 2.0                # box half width in time per unit row gap (cm)
    pair_c2: float = 0.2              # pair score acceptance (cm^2)
    max_gap: int = 2
    min_track_hits: int = 10
    bz: float = 0.5                   # tesla
    sigma_y: float = 0.1              # cm
    sigma_t: float = 0.1              # cm
    var_s: float | None = 1.0         # prior variances (None = prior off)
    var_tau: float | None = 1.0
    var_k: float | None = 100.0       # (1/GeV)^2
    max_iter: int = 50
    s_max: float = 0.999

    def _c(self):
        self._rx = np.ascontiguousarray(self.row_x, np.float32)
        c = _Cfg()
        c.n_rows = len(self._rx)
        c.row_x = self._rx.ctypes.data
        c.win_y, c.win_t, c.pair_c2 = self.win_y, self.win_t, self.pair_c2
        c.max_gap, c.min_track_hits = self.max_gap, self.min_track_hits
        c.bz, c.sigma_y, c.sigma_t = self.bz, self.sigma_y, self.sigma_t
        c.ivar_s = 0.0 if self.var_s is None else 1.0 / self.var_s
        c.ivar_tau = 0.0 if self.var_tau is None else 1.0 / self.var_tau
        c.ivar_k = 0.0 if self.var_k is None else 1.0 / self.var_k
        c.max_iter, c.s_max = self.max_iter, self.s_max
        return c


def _p(a):
    return a.ctypes.data


def _in(row, y, t):
    return (np.ascontiguousarray(row, np.uint8), np.ascontiguousarray(y, np.float32),
            np.ascontiguousarray(t, np.float32))


def links(cfg: Config, row, y, t):
    """Uncleaned links (up, dn, gap) of every hit, in input-index space."""
    lib = _load()
    row, y, t = _in(row, y, t)
    n = len(row)
    up = np.empty(n, np.int32); dn = np.empty(n, np.int32); gap = np.empty(n, np.int32)
    c = cfg._c()
    lib.ora_links(ctypes.byref(c), n, _p(row), _p(y), _p(t), _p(up), _p(dn), _p(gap))
    return up, dn, gap


def links_subset(cfg: Config, row, y, t, query):
    """Uncleaned links of the listed hits only (indexed like `query`)."""
    lib = _load()
    row, y, t = _in(row, y, t)
    q = np.ascontiguousarray(query, np.int32)
    up = np.empty(len(q), np.int32); dn = np.empty(len(q), np.int32); gap = np.empty(len(q), np.int32)
    c = cfg._c()
    lib.ora_links_subset(ctypes.byref(c), len(row), _p(row), _p(y), _p(t), len(q), _p(q), _p(up), _p(dn), _p(gap))
    return up, dn, gap


def clean(up, dn):
    lib = _load()
    up = np.ascontiguousarray(up, np.int32); dn = np.ascontiguousarray(dn, np.int32)
    upc = np.empty_like(up); dnc = np.empty_like(dn)
    lib.ora_clean(len(up), _p(up), _p(dn), _p(upc), _p(dnc))
    return upc, dnc


def tracks(cfg: Config, upc, dnc):
    """Tracks from cleaned links: (first int64[T], len int32[T], clusters int32[], assign int32[n])."""
    lib = _load()
    upc = np.ascontiguousarray(upc, np.int32); dnc = np.ascontiguousarray(dnc, np.int32)
    n = len(upc)
    first = np.empty(max(n, 1), np.int64); ln = np.empty(max(n, 1), np.int32)
    cl = np.empty(max(n, 1), np.int32); assign = np.empty(n, np.int32)
    c = cfg._c()
    nt = lib.ora_tracks(ctypes.byref(c), n, _p(upc), _p(dnc), _p(first), _p(ln), _p(cl), _p(assign))
    nc = int(ln[:nt].sum()) if nt else 0
    return first[:nt].copy(), ln[:nt].copy(), cl[:nc].copy(), assign


def chain_len(upc, dnc):
    lib = _load()
    upc = np.ascontiguousarray(upc, np.int32); dnc = np.ascontiguousarray(dnc, np.int32)
    out = np.empty(len(upc), np.int32)
    lib.ora_chain_len(len(upc), _p(upc), _p(dnc), _p(out))
    return out


def fit_map(cfg: Config, x, y, t):
    """FP64 MAP helix fit of one track (clusters ordered by row)."""
    lib = _load()
    x = np.ascontiguousarray(x, np.float64); y = np.ascontiguousarray(y, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    out = np.zeros(1, FIT_DTYPE)
    c = cfg._c()
    lib.ora_fit_map(ctypes.byref(c), len(x), _p(x), _p(y), _p(t), _p(out))
    return out[0]


def fit_kf(cfg: Config, x, y, t, passes: int = 3):
    """FP64 Kalman diagnostic (pass 1 extended, then linearised passes)."""
    lib = _load()
    x = np.ascontiguousarray(x, np.float64); y = np.ascontiguousarray(y, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    out = np.zeros(1, FIT_DTYPE)
    c = cfg._c()
    lib.ora_fit_kf(ctypes.byref(c), len(x), _p(x), _p(y), _p(t), passes, _p(out))
    return out[0]


def map_cost(cfg: Config, x, y, t, q, q0):
    lib = _load()
    x = np.ascontiguousarray(x, np.float64); y = np.ascontiguousarray(y, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    q = np.ascontiguousarray(q, np.float64); q0 = np.ascontiguousarray(q0, np.float64)
    c = cfg._c()
    return lib.ora_map_cost(ctypes.byref(c), len(x), _p(x), _p(y), _p(t), _p(q), _p(q0))


def propagate(cfg: Config, q, dx):
    """Closed-form helix transport of state q=(y,t,sinphi,tau,q/pT) by dx; (q', F) or None."""
    lib = _load()
    q = np.ascontiguousarray(q, np.float64)
    qo = np.zeros(5); F = np.zeros(25)
    c = cfg._c()
    ok = lib.ora_propagate_c(ctypes.byref(c), _p(q), float(dx), _p(qo), _p(F))
    return (qo, F.reshape(5, 5)) if ok else None


def fit_tracks(cfg: Config, first, ln, clusters, row, y, t, kf_passes: int = 0):
    """Fit every track of a sector: MAP (kf_passes=0) or the Kalman diagnostic."""
    lib = _load()
    row, y, t = _in(row, y, t)
    first = np.ascontiguousarray(first, np.int64); ln = np.ascontiguousarray(ln, np.int32)
    clusters = np.ascontiguousarray(clusters, np.int32)
    out = np.zeros(len(first), FIT_DTYPE)
    c = cfg._c()
    if len(first):
        lib.ora_fit_tracks(ctypes.byref(c), len(first), _p(first), _p(ln), _p(clusters), _p(row), _p(y), _p(t),
                           kf_passes, _p(out))
    return out


class _FollowCfg(ctypes.Structure):
    _fields_ = [("win_y", ctypes.c_float), ("win_t", ctypes.c_float), ("chi2_max", ctypes.c_float),
                ("q_slope", ctypes.c_float), ("var_y", ctypes.c_float), ("var_t", ctypes.c_float),
                ("var_slope0", ctypes.c_float), ("max_miss", ctypes.c_int32)]


@dataclass
class FollowConfig:
    """Constants of the track following (the readings adopted for this build)."""
    win_y: float = 1.5          # search box half widths around the prediction (cm)
    win_t: float = 1.5
    chi2_max: float = 16.0      # gate on dy^2/Vy + dt^2/Vt
    q_slope: float = 1e-4       # slope variance added per cm of |dx|
    var_y: float = 0.01         # measurement variances (cm^2)
    var_t: float = 0.01
    var_slope0: float = 1.0     # initial slope variance
    max_miss: int = 3           # consecutive rows without a cluster that end an extension

    def _c(self):
        c = _FollowCfg()
        for k in ("win_y", "win_t", "chi2_max", "q_slope", "var_y", "var_t", "var_slope0", "max_miss"):
            setattr(c, k, getattr(self, k))
        return c


def follow(cfg: Config, fcfg: FollowConfig, row, y, t, first, ln, clusters):
    """Track following and selection of one sector's tracks: the kept tracks
    (first, len, clusters), the assignment, and per input track the inward
    and outward extension counts and the kept cluster count (-1: dropped)."""
    lib = _load()
    row, y, t = _in(row, y, t)
    first = np.ascontiguousarray(first, np.int64); ln = np.ascontiguousarray(ln, np.int32)
    clusters = np.ascontiguousarray(clusters, np.int32)
    n, nt = len(row), len(first)
    of = np.empty(max(nt, 1), np.int64); ol = np.empty(max(nt, 1), np.int32)
    oc = np.empty(max(n, 1), np.int32); assign = np.empty(n, np.int32)
    ei = np.zeros(max(nt, 1), np.int32); eo = np.zeros(max(nt, 1), np.int32); kept = np.zeros(max(nt, 1), np.int32)
    c = cfg._c()
    fc = fcfg._c()
    k = lib.ora_follow(ctypes.byref(c), ctypes.byref(fc), n, _p(row), _p(y), _p(t), nt, _p(first), _p(ln),
                       _p(clusters), _p(of), _p(ol), _p(oc), _p(assign), _p(ei), _p(eo), _p(kept))
    nc = int(ol[:k].sum()) if k else 0
    return dict(first=of[:k].copy(), len=ol[:k].copy(), clusters=oc[:nc].copy(), assign=assign,
                ext_in=ei[:nt].copy(), ext_out=eo[:nt].copy(), kept=kept[:nt].copy())


def kf1_run(x, m, var, var_slope0, q):
    """The following's 1-D filter over the points (x, m) in order, started at
    the first: (value, slope, p00, p01, p11) at the last point."""
    lib = _load()
    x = np.ascontiguousarray(x, np.float32); m = np.ascontiguousarray(m, np.float32)
    out = np.zeros(5, np.float32)
    lib.ora_kf1_run(len(x), _p(x), _p(m), var, var_slope0, q, _p(out))
    return out


def run_sector(cfg: Config, row, y, t, fit: bool = True, follow_cfg: FollowConfig | None = None):
    """The whole path on one sector: links, cleaning, chains, assignment, fit."""
    up, dn, gap = links(cfg, row, y, t)
    upc, dnc = clean(up, dn)
    first, ln, cl, assign = tracks(cfg, upc, dnc)
    res = dict(up=up, dn=dn, gap=gap, upc=upc, dnc=dnc, first=first, len=ln, clusters=cl, assign=assign)
    if follow_cfg is not None:
        fo = follow(cfg, follow_cfg, row, y, t, first, ln, cl)
        res["chains"] = dict(first=first, len=ln, clusters=cl, assign=assign)
        res.update(first=fo["first"], len=fo["len"], clusters=fo["clusters"], assign=fo["assign"],
                   ext_in=fo["ext_in"], ext_out=fo["ext_out"], kept=fo["kept"])
        first, ln, cl = fo["first"], fo["len"], fo["clusters"]
    if fit:
        res["fit"] = fit_tracks(cfg, first, ln, cl, row, y, t)
    return res


# ------------------------------------------------------ collision time
DRIFT_LENGTH = 250.0   # cm: t = v_d t_coll + (drift length - |z|) (R2)


def track_t0(cfg: Config, x_ref, y, t, sinphi, tau, qpt):
    """Collision time of a track in drift cm (R28): the drift time of its
    helix at the point of closest approach to the beam line in the
    transverse plane, minus the drift length. From the state at x_ref
    (position (x_ref, y), direction (cos phi, sin phi), curvature
    kappa = -kB q/pT) the signed arc length s to that point solves
    r(s) . r'(s) = 0 on the circle, tan(kappa s) = -a kappa / (1 + b kappa)
    with a = r . direction and b = r . left normal (the root nearest to the
    state: s = -a for a straight track); the time there is t + tau s. For a
    track of one side (z of one sign) this is v_d t_coll - z_vertex on the A
    side and v_d t_coll + z_vertex on the C side. FP64."""
    x = np.asarray(x_ref, np.float64); yy = np.asarray(y, np.float64)
    s = np.asarray(sinphi, np.float64); k = -2.99792458e-3 * cfg.bz * np.asarray(qpt, np.float64)
    c = np.sqrt(1.0 - s * s)
    a = x * c + yy * s
    b = -x * s + yy * c
    with np.errstate(divide="ignore", invalid="ignore"):
        sd = np.where(k != 0.0, np.arctan2(-a * k, 1.0 + b * k) / np.where(k != 0.0, k, 1.0), -a)
    return np.asarray(t, np.float64) + np.asarray(tau, np.float64) * sd - DRIFT_LENGTH


def collision_groups(t0, gap: float):
    """Collision candidates of one side of a frame (R29): the tracks in
    ascending t0, a new group wherever the next t0 exceeds the previous by
    more than gap. Group numbers in ascending t0; returns int32 per track."""
    t0 = np.asarray(t0, np.float64)
    out = np.zeros(len(t0), np.int32)
    if len(t0) == 0:
        return out
    order = np.argsort(t0, kind="stable")
    v = t0[order]
    new = np.concatenate([[False], (v[1:] - v[:-1]) > gap])
    out[order] = np.cumsum(new).astype(np.int32)
    return out


def collision_assign(t0, n_clusters, gap: float, min_clusters: int, window: float):
    """Collision candidates of one side of a frame with the tracks attached
    to them (R29). Anchors are the tracks of at least min_clusters clusters
    with a finite t0; they alone form the groups (collision_groups over the
    anchors), and a group's time is the mean t0 of its anchors. Every other
    track with a finite t0 joins the group whose time is nearest (the earlier
    one on a tie) if that distance is at most window.

    Returns (group per track, -1 for none; group times; anchors per group;
    tracks per group)."""
    t0 = np.asarray(t0, np.float64)
    n_clusters = np.asarray(n_clusters)
    group = np.full(len(t0), -1, np.int32)
    fin = np.isfinite(t0)
    anchor = fin & (n_clusters >= min_clusters)
    ia = np.nonzero(anchor)[0]
    if len(ia) == 0:
        return group, np.zeros(0), np.zeros(0, np.int64), np.zeros(0, np.int64)
    ga = collision_groups(t0[ia], gap)
    group[ia] = ga
    ng = int(ga.max()) + 1
    n_anchor = np.bincount(ga, minlength=ng).astype(np.int64)
    mean = np.bincount(ga, t0[ia], ng) / n_anchor
    io = np.nonzero(fin & ~anchor)[0]
    if len(io):
        v = t0[io]
        j = np.searchsorted(mean, v)
        lo = np.clip(j - 1, 0, ng - 1)
        hi = np.clip(j, 0, ng - 1)
        d_lo, d_hi = np.abs(v - mean[lo]), np.abs(v - mean[hi])
        near = np.where(d_lo <= d_hi, lo, hi)
        dist = np.minimum(d_lo, d_hi)
        group[io] = np.where(dist <= window, near, -1)
    n_all = np.bincount(group[group >= 0], minlength=ng).astype(np.int64)
    return group, mean, n_anchor, n_all


# ---------------------------------------------------- sector merging
MERGE_SIGMA = (0.5, 0.02, 0.5, 0.01)   # transverse miss (cm), direction (rad), time (cm), tau


def sector_alpha(sector: int) -> float:
    """Azimuth of a sector's centre (the local x axis): sectors k and k + 18
    (A and C side) at ((k mod 18) + 1/2) 20 degrees."""
    return ((sector % 18) + 0.5) * np.deg2rad(20.0)


def merge_residuals(cfg: Config, A, B, dalpha: float):
    """Residuals (R30) of track state B seen from the helix of track A, for
    all pairs (rows A, columns B): B's reference point and direction are
    rotated into A's frame (B's sector lies dalpha further in azimuth); on
    A's circle (direction phi_A, curvature kappa = -kB q/pT) the point
    nearest to B's lies at the turning angle theta = atan2(kappa a,
    1 - kappa b), where (a, b) is B's point relative to A's along and across
    A's direction, i.e. at transverse arc theta / kappa (a for a straight
    track). Returned: the signed transverse miss (2 b - kappa (a^2 + b^2)) /
    (1 + sqrt((kappa a)^2 + (1 - kappa b)^2)) (b for a straight track), B's
    direction minus A's there (wrapped to (-pi, pi]), A's time there minus
    B's, and tau_A - tau_B. A and B: dicts of x, y, t, sinphi, tau, qpt. FP64."""
    ax, ay, at = (np.asarray(A[k], np.float64) for k in ("x", "y", "t"))
    asp, atau, aq = (np.asarray(A[k], np.float64) for k in ("sinphi", "tau", "qpt"))
    bx, by, bt = (np.asarray(B[k], np.float64) for k in ("x", "y", "t"))
    bsp, btau = (np.asarray(B[k], np.float64) for k in ("sinphi", "tau"))
    ca = np.sqrt(1.0 - asp * asp)
    xb = bx * np.cos(dalpha) - by * np.sin(dalpha)
    yb = bx * np.sin(dalpha) + by * np.cos(dalpha)
    vx = xb[None, :] - ax[:, None]
    vy = yb[None, :] - ay[:, None]
    a = vx * ca[:, None] + vy * asp[:, None]
    b = -vx * asp[:, None] + vy * ca[:, None]
    k = (-2.99792458e-3 * cfg.bz * aq)[:, None]
    th = np.arctan2(k * a, 1.0 - k * b)
    with np.errstate(divide="ignore", invalid="ignore"):
        arc = np.where(k != 0.0, th / np.where(k != 0.0, k, 1.0), a)
    h = np.sqrt((k * a) ** 2 + (1.0 - k * b) ** 2)
    dr = (2.0 * b - k * (a * a + b * b)) / (1.0 + h)
    dphi = np.arcsin(bsp)[None, :] + dalpha - (np.arcsin(asp)[:, None] + th)
    dphi = np.arctan2(np.sin(dphi), np.cos(dphi))
    dt = at[:, None] + atau[:, None] * arc - bt[None, :]
    dtau = atau[:, None] - btau[None, :]
    return dr, dphi, dt, dtau


def merge_sectors(cfg: Config, tracks, min_clusters: int = 30, window: float = 8.0, d2_cut: float = 25.0,
                  sectors=None):
    """Sector merging of one frame (R30). tracks[s] for s = 0..35: dict of
    the fitted parameters (x, y, t = fitted time at x, sinphi, tau, qpt),
    status, n (clusters) and t0 of the sector's tracks. Eligible: status 0,
    at least min_clusters clusters, finite t0. Sector k + 18 side has the
    next sector (k + 1) mod 18 + 18 side, 20 degrees further. A pair
    (A in s, B in next(s)) with |t0_A - t0_B| <= window is scored with
    D2 = sum (residual / MERGE_SIGMA)^2 of merge_residuals(A, B) and is a
    candidate if D2 <= d2_cut; it is merged if B is A's best candidate and A
    is B's (least D2, then least index). Returns, per sector, int32 arrays
    (next partner index in next(s), previous partner index in prev(s), -1
    for none) and the D2 of each merged pair. sectors: only the pairs (s, next(s)) for s in it
    (default: all)."""
    sig = np.asarray(MERGE_SIGMA, np.float64)
    nxt = [np.full(len(tracks[s]["status"]), -1, np.int32) for s in range(36)]
    prv = [np.full(len(tracks[s]["status"]), -1, np.int32) for s in range(36)]
    d2_pairs = []
    for s in (range(36) if sectors is None else sectors):
        side, kk = divmod(s, 18)
        n = 18 * side + (kk + 1) % 18
        A, B = tracks[s], tracks[n]
        ea = np.nonzero((np.asarray(A["status"]) == 0) & (np.asarray(A["n"]) >= min_clusters)
                        & np.isfinite(np.asarray(A["t0"], np.float64)))[0]
        eb = np.nonzero((np.asarray(B["status"]) == 0) & (np.asarray(B["n"]) >= min_clusters)
                        & np.isfinite(np.asarray(B["t0"], np.float64)))[0]
        if len(ea) == 0 or len(eb) == 0:
            continue
        sub = lambda T, e: {k: np.asarray(T[k], np.float64)[e] for k in ("x", "y", "t", "sinphi", "tau", "qpt", "t0")}
        a, b = sub(A, ea), sub(B, eb)
        d2 = np.full((len(ea), len(eb)), np.inf)
        for i0 in range(0, len(ea), 512):   # bounded memory
            i1 = min(i0 + 512, len(ea))
            r = merge_residuals(cfg, {k: v[i0:i1] for k, v in a.items()}, b, np.deg2rad(20.0))
            v = sum((ri / si) ** 2 for ri, si in zip(r, sig))
            near = np.abs(a["t0"][i0:i1, None] - b["t0"][None, :]) <= window
            d2[i0:i1] = np.where(near & (v <= d2_cut), v, np.inf)
        # best per row and per column: least D2, then least index (argmin takes the first)
        best_b = np.argmin(d2, axis=1)
        best_a = np.argmin(d2, axis=0)
        for i in range(len(ea)):
            j = best_b[i]
            if np.isfinite(d2[i, j]) and best_a[j] == i:
                nxt[s][ea[i]] = eb[j]
                prv[n][eb[j]] = ea[i]
                d2_pairs.append(d2[i, j])
    return nxt, prv, np.asarray(d2_pairs)



MEMBRANE_S_MARGIN = 5.0  # arc margin (cm) of the crossing test
MEMBRANE_S_TOL = 1.0     # time tolerance (cm) of that test


def ref_arc(cfg: Config, x_ref, y, sinphi, qpt):
    """Transverse arc from the point of closest approach to the beam line to
    the state at (x_ref, y) (minus the arc of track_t0). FP64."""
    x = np.asarray(x_ref, np.float64); yy = np.asarray(y, np.float64)
    s = np.asarray(sinphi, np.float64); k = -2.99792458e-3 * cfg.bz * np.asarray(qpt, np.float64)
    c = np.sqrt(1.0 - s * s)
    a = x * c + yy * s
    b = -x * s + yy * c
    with np.errstate(divide="ignore", invalid="ignore"):
        sd = np.where(k != 0.0, np.arctan2(-a * k, 1.0 + b * k) / np.where(k != 0.0, k, 1.0), -a)
    return -sd


def membrane_residuals(cfg: Config, A, B):
    """Residuals (Sec. 1, reading R32) of track state B (sector k + 18, C side) seen from
    the helix of track A (sector k, A side, the same azimuth): the transverse
    miss and direction difference at the point of A's circle nearest to B's
    (merge_residuals with no rotation), and tau_A + tau_B (the drift time
    runs against z on the A side and with it on the C side, so one
    particle's two pieces have opposite tau). Also returns whether the
    particle's crossing of z = 0 lies between the pieces: the two time lines
    t0 + tau s (s the transverse arc from the beam line) agree within
    MEMBRANE_S_TOL cm at some s from the inner piece's reference arc (the
    smaller of the two, ref_arc) to the outer piece's, widened by
    MEMBRANE_S_MARGIN cm at both ends. All pairs (rows A, columns B). FP64."""
    dr, dphi, _, _ = merge_residuals(cfg, A, B, 0.0)
    atau = np.asarray(A["tau"], np.float64)[:, None]
    btau = np.asarray(B["tau"], np.float64)[None, :]
    dtau = atau + btau
    dT = np.asarray(B["t0"], np.float64)[None, :] - np.asarray(A["t0"], np.float64)[:, None]
    sa = ref_arc(cfg, A["x"], A["y"], A["sinphi"], A["qpt"])[:, None]
    sb = ref_arc(cfg, B["x"], B["y"], B["sinphi"], B["qpt"])[None, :]
    s_lo = np.minimum(sa, sb) - MEMBRANE_S_MARGIN
    s_hi = np.maximum(sa, sb) + MEMBRANE_S_MARGIN
    D = atau - btau
    meet = (dT >= np.minimum(D * s_lo, D * s_hi) - MEMBRANE_S_TOL) & (dT <= np.maximum(D * s_lo, D * s_hi) + MEMBRANE_S_TOL)
    return dr, dphi, dtau, meet


def merge_membrane(cfg: Config, tracks, min_clusters: int = 30, window: float = 30.0, d2_cut: float = 25.0,
                   sectors=None):
    """Membrane merging of one frame (Sec. 1, reading R32): a pair (A in sector k of the A
    side, B in sector k + 18) with both eligible as in merge_sectors,
    |t0_A - t0_B| <= window (the two pieces' collision times differ by twice
    the vertex z) and time lines that meet between the pieces is scored
    with D2 = (dr / 0.5)^2 + (dphi / 0.02)^2 + (dtau / 0.01)^2 of
    membrane_residuals; candidates have D2 <= d2_cut; a pair is merged if
    each is the other's best (least D2, then least index). Returns, per
    sector, int32 arrays of the partner's index in the other side's sector
    (-1: none), and the D2 of each merged pair. sectors: only the pairs
    (k, k + 18) for k in it (default: 0..17)."""
    sig = np.asarray(MERGE_SIGMA, np.float64)
    part = [np.full(len(tracks[s]["status"]), -1, np.int32) for s in range(36)]
    d2_pairs = []
    el = lambda T: np.nonzero((np.asarray(T["status"]) == 0) & (np.asarray(T["n"]) >= min_clusters)
                              & np.isfinite(np.asarray(T["t0"], np.float64)))[0]
    for s in (range(18) if sectors is None else sectors):
        A, B = tracks[s], tracks[s + 18]
        ea, eb = el(A), el(B)
        if len(ea) == 0 or len(eb) == 0:
            continue
        sub = lambda T, e: {k: np.asarray(T[k], np.float64)[e] for k in ("x", "y", "t", "sinphi", "tau", "qpt", "t0")}
        a, b = sub(A, ea), sub(B, eb)
        d2 = np.full((len(ea), len(eb)), np.inf)
        for i0 in range(0, len(ea), 512):
            i1 = min(i0 + 512, len(ea))
            dr, dphi, dtau, meet = membrane_residuals(cfg, {k: v[i0:i1] for k, v in a.items()}, b)
            v = (dr / sig[0]) ** 2 + (dphi / sig[1]) ** 2 + (dtau / sig[3]) ** 2
            near = np.abs(a["t0"][i0:i1, None] - b["t0"][None, :]) <= window
            d2[i0:i1] = np.where(near & meet & (v <= d2_cut), v, np.inf)
        best_b = np.argmin(d2, axis=1)
        best_a = np.argmin(d2, axis=0)
        for i in range(len(ea)):
            j = best_b[i]
            if np.isfinite(d2[i, j]) and best_a[j] == i:
                part[s][ea[i]] = eb[j]
                part[s + 18][eb[j]] = ea[i]
                d2_pairs.append(d2[i, j])
    return part, np.asarray(d2_pairs)


def refit_merged(cfg: Config, xa, ya, ta, xb, yb, tb, dalpha: float):
    """Global refit of a merged pair (Sec. 1 and Sec. 3, reading R31): the clusters of the second track
    (in the sector dalpha further in azimuth) rotated into the first track's
    frame, appended to the first track's, ordered by local x (a stable sort:
    ties keep that order), and fitted by fit_map as one track. FP64."""
    xa, ya, ta, xb, yb, tb = (np.asarray(v, np.float64) for v in (xa, ya, ta, xb, yb, tb))
    c, s = np.cos(dalpha), np.sin(dalpha)
    x = np.concatenate([xa, xb * c - yb * s])
    y = np.concatenate([ya, xb * s + yb * c])
    t = np.concatenate([ta, tb])
    o = np.argsort(x, kind="stable")
    return fit_map(cfg, x[o], y[o], t[o])


def remove_clusters(n_clusters: int, assign, status, qpt, pt_min: float):
    """Removal of the clusters of tracks not used for physics (Sec. 1, reading R33), one
    sector: the input indices kept, ascending. A cluster is removed if its
    track (assign: the sector's track number per input cluster, -1 for none)
    has a successful fit (status 0) and a transverse momentum below pt_min
    (|q/pT| > 1 / pt_min); clusters of no track, and of tracks whose fit
    failed, are kept."""
    assign = np.asarray(assign, np.int64)
    status = np.asarray(status)
    qpt = np.asarray(qpt, np.float64)
    assert len(assign) == n_clusters
    low = (status == 0) & (np.abs(qpt) > 1.0 / pt_min)
    removed = np.zeros(n_clusters, bool)
    on = assign >= 0
    removed[on] = low[assign[on]]
    return np.nonzero(~removed)[0].astype(np.int32)


ENT_Q = 16.0        # quantisation: 1/16 cm
ENT_H = 255         # symbols in [-ENT_H, ENT_H] have a bin; the rest share the escape bin
ENT_BINS = 2 * ENT_H + 2
ENT_STREAMS = 5     # row step; y, t first differences; y, t track-model residuals


def entropy_symbols(row, y, t):
    """Symbols of one track's clusters (rows ascending) for the entropy
    reduction (Sec. 1, reading R34). Coordinates are quantised to 1/16 cm (FP32 product,
    rounded to nearest even). Every cluster after the first gives: the row
    step dr_j; the first differences of y and t; and the track-model
    residuals of y and t: the first difference for the second cluster, and
    from the third on the exact integer q_j dr_{j-1} - q_{j-1} (dr_{j-1} +
    dr_j) + q_{j-2} dr_j (dr_{j-1} times the miss of the straight-line
    extrapolation in row number). Returns int64 [n - 1, 5]."""
    r = np.asarray(row, np.int64)
    qy = np.rint(np.asarray(y, np.float32) * np.float32(ENT_Q)).astype(np.int64)
    qt = np.rint(np.asarray(t, np.float32) * np.float32(ENT_Q)).astype(np.int64)
    n = len(r)
    out = np.zeros((max(n - 1, 0), ENT_STREAMS), np.int64)
    for j in range(1, n):
        dr = r[j] - r[j - 1]
        out[j - 1, 0] = dr
        out[j - 1, 1] = qy[j] - qy[j - 1]
        out[j - 1, 2] = qt[j] - qt[j - 1]
        if j == 1:
            out[j - 1, 3] = qy[j] - qy[j - 1]
            out[j - 1, 4] = qt[j] - qt[j - 1]
        else:
            dp = r[j - 1] - r[j - 2]
            out[j - 1, 3] = qy[j] * dp - qy[j - 1] * (dp + dr) + qy[j - 2] * dr
            out[j - 1, 4] = qt[j] * dp - qt[j - 1] * (dp + dr) + qt[j - 2] * dr
    return out


def entropy_histograms(first, ln, clusters, row, y, t):
    """Histograms [5, ENT_BINS] of the symbols of every track of a sector
    (symbol s in bin s + ENT_H if |s| <= ENT_H, else the last bin)."""
    h = np.zeros((ENT_STREAMS, ENT_BINS), np.int64)
    row = np.asarray(row); y = np.asarray(y, np.float32); t = np.asarray(t, np.float32)
    for f0, L in zip(first, ln):
        c = clusters[f0:f0 + L]
        sym = entropy_symbols(row[c], y[c], t[c])
        b = np.where(np.abs(sym) <= ENT_H, sym + ENT_H, ENT_BINS - 1)
        for k in range(ENT_STREAMS):
            h[k] += np.bincount(b[:, k], minlength=ENT_BINS)
    return h


def entropy_bits(h, escape_bits: float = 32.0):
    """Order-0 entropy in bits of each stream's symbols (an escape costs its
    bin's code plus escape_bits)."""
    h = np.asarray(h, np.float64)
    out = []
    for k in range(h.shape[0]):
        n = h[k].sum()
        p = h[k][h[k] > 0] / max(n, 1.0)
        out.append(float(-(h[k][h[k] > 0] * np.log2(p)).sum() + escape_bits * h[k][-1]))
    return np.asarray(out)


ANS_BITS = 16              # frequencies of a model sum to 2^16
ANS_L = 1 << 23            # the coder's state stays in [2^23, 2^31)
ANS_STREAMS = (0, 3, 4)    # coded: the row step and the track-model residuals (the rest follows from them)


def ans_model(h):
    """Frequencies (sum 2^16, every bin with a count >= 1) of one stream's
    histogram for the rANS coder (R35): f = max(1, floor(count 2^16 /
    total)) for counted bins; the shortfall is added to the bin of the
    largest count (lowest index on ties), an excess taken one unit at a
    time from the bin of the largest frequency (lowest index on ties).
    Bins without a count get 0; the escape bin always gets at least 1.
    Returns int64 frequencies and cumulative starts."""
    h = np.asarray(h, np.int64).copy()
    h[-1] = max(h[-1], 1)
    tot = int(h.sum())
    M = 1 << ANS_BITS
    f = np.where(h > 0, np.maximum(1, (h * M) // tot), 0)
    d = M - int(f.sum())
    if d > 0:
        f[int(np.argmax(h))] += d
    while d < 0:
        i = int(np.argmax(f))
        f[i] -= 1
        d += 1
    c = np.concatenate([[0], np.cumsum(f)[:-1]])
    return f, c


def _ans_put(x, f, c, out):
    xmax = ((ANS_L >> ANS_BITS) << 8) * f
    while x >= xmax:
        out.append(x & 255)
        x >>= 8
    return ((x // f) << ANS_BITS) + (x % f) + c


def ans_encode_track(sym, models):
    """rANS bytes of one track's symbols (rows of entropy_symbols; the
    streams ANS_STREAMS are coded, the first differences following from
    them): one state, the clusters' symbols coded last to first so that a
    decoder reads them first to last; each symbol through its stream's model, a symbol
    beyond +-ENT_H as the escape bin followed by its value as two uniform
    16-bit parts. Returns the bytes in decoding order (the final state, 4
    bytes little end last, first)."""
    x = ANS_L
    out = []
    for row in np.asarray(sym, np.int64)[::-1]:
        for k in ANS_STREAMS[::-1]:
            v = int(row[k])
            f, c = models[k]
            if abs(v) <= ENT_H:
                x = _ans_put(x, int(f[v + ENT_H]), int(c[v + ENT_H]), out)
            else:
                u = v & 0xFFFFFFFF
                x = _ans_put(x, 1, u & 0xFFFF, out)          # low half (decoded last)
                x = _ans_put(x, 1, u >> 16, out)             # high half
                x = _ans_put(x, int(f[-1]), int(c[-1]), out)
    for _ in range(4):
        out.append(x & 255)
        x >>= 8
    return bytes(reversed(out))


def ans_decode_track(data, n, models):
    """Inverse of ans_encode_track for n clusters' symbols: int64 [n, 5]
    with the coded streams filled (the others zero)."""
    data = bytes(data)
    x, p = 0, 0
    for _ in range(4):
        x = (x << 8) | data[p]
        p += 1
    M = (1 << ANS_BITS) - 1

    def get(f, c):
        nonlocal x, p
        s = x & M
        i = int(np.searchsorted(c, s, side="right") - 1)
        x = int(f[i]) * (x >> ANS_BITS) + s - int(c[i])
        while x < ANS_L:
            x = (x << 8) | data[p]
            p += 1
        return i

    def get_raw():
        nonlocal x, p
        s = x & M
        x = (x >> ANS_BITS)
        while x < ANS_L:
            x = (x << 8) | data[p]
            p += 1
        return s

    out = np.zeros((n, ENT_STREAMS), np.int64)
    for j in range(n):
        for k in ANS_STREAMS:
            f, c = models[k]
            i = get(f, c)
            if i == ENT_BINS - 1:
                hi = get_raw()
                lo = get_raw()
                u = (hi << 16) | lo
                out[j, k] = u - (1 << 32) if u >= (1 << 31) else u
            else:
                out[j, k] = i - ENT_H
    assert p == len(data)
    return out

# ----------------------------------------------------------------- MLP
MLP_IN, MLP_INP, MLP_H = 12, 16, 64
MLP_NPARAM = MLP_H * MLP_INP + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1


def bf16(a):
    """Round float32 values to BF16 (nearest even), returned as float32."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    special = (u & 0x7F800000) == 0x7F800000
    r = np.where(special, (u & 0xFFFF0000).astype(np.uint32) | np.where((u & 0x7FFFFF) != 0, 0x400000, 0), r)
    return r.astype(np.uint32).view(np.float32).reshape(a.shape)


@dataclass
class MLP:
    """Network weights (FP32 values on the BF16 grid for w*, FP32 biases)."""
    w1: np.ndarray   # [64, 16] (columns 12..15 unused, zero)
    b1: np.ndarray   # [64]
    w2: np.ndarray   # [64, 64]
    b2: np.ndarray   # [64]
    w3: np.ndarray   # [64]
    b3: float

    def flat(self):
        return np.concatenate([np.asarray(self.w1, np.float32).ravel(), np.asarray(self.b1, np.float32),
                               np.asarray(self.w2, np.float32).ravel(), np.asarray(self.b2, np.float32),
                               np.asarray(self.w3, np.float32), np.array([self.b3], np.float32)])

    @staticmethod
    def from_flat(v):
        v = np.asarray(v, np.float32)
        o = 0
        def take(n):
            nonlocal o
            r = v[o:o + n]
            o += n
            return r
        w1 = take(MLP_H * MLP_INP).reshape(MLP_H, MLP_INP); b1 = take(MLP_H)
        w2 = take(MLP_H * MLP_H).reshape(MLP_H, MLP_H); b2 = take(MLP_H)
        w3 = take(MLP_H); b3 = float(take(1)[0])
        return MLP(w1.copy(), b1.copy(), w2.copy(), b2.copy(), w3.copy(), b3)

    @staticmethod
    def random(seed=0, scale=1.0):
        rng = np.random.default_rng(seed)
        w1 = np.zeros((MLP_H, MLP_INP), np.float32)
        w1[:, :MLP_IN] = rng.normal(0, scale * np.sqrt(2.0 / MLP_IN), (MLP_H, MLP_IN))
        w2 = rng.normal(0, scale * np.sqrt(2.0 / MLP_H), (MLP_H, MLP_H))
        w3 = rng.normal(0, scale * np.sqrt(1.0 / MLP_H), MLP_H)
        return MLP(bf16(w1), rng.normal(0, 0.1, MLP_H).astype(np.float32), bf16(w2),
                   rng.normal(0, 0.1, MLP_H).astype(np.float32), bf16(w3), 0.0)


def mlp_forward(m: MLP, x, round_act=True):
    lib = _load()
    x = np.ascontiguousarray(x, np.float32).reshape(-1, MLP_INP)
    z = np.zeros(len(x), np.float64)
    w = m.flat()
    lib.ora_mlp_forward_batch(_p(w), len(x), _p(x), 1 if round_act else 0, _p(z))
    return z


def mlp_grad(m: MLP, x, label, w_pos=1.0, round_act=True):
    """Mean weighted BCE-with-logits loss and its FP64 gradient (an MLP of
    gradients, as float64 arrays)."""
    lib = _load()
    x = np.ascontiguousarray(x, np.float32).reshape(-1, MLP_INP)
    lab = np.ascontiguousarray(label, np.float32)
    g1 = np.zeros((MLP_H, MLP_INP)); gb1 = np.zeros(MLP_H); g2 = np.zeros((MLP_H, MLP_H)); gb2 = np.zeros(MLP_H)
    g3 = np.zeros(MLP_H); gb3 = np.zeros(1)
    w = m.flat()
    loss = lib.ora_mlp_grad(_p(w), len(x), _p(x), _p(lab), float(w_pos), 1 if round_act else 0,
                            _p(g1), _p(gb1), _p(g2), _p(gb2), _p(g3), _p(gb3))
    return loss, dict(w1=g1, b1=gb1, w2=g2, b2=gb2, w3=g3, b3=gb3[0])


def decay_mask():
    """1 for the weights (w1, w2, w3), 0 for the biases, in the flat
    parameter order: AdamW decays the weights only."""
    m = np.zeros(MLP_NPARAM, np.uint8)
    m[:MLP_H * MLP_INP] = 1
    o = MLP_H * MLP_INP + MLP_H
    m[o:o + MLP_H * MLP_H] = 1
    o += MLP_H * MLP_H + MLP_H
    m[o:o + MLP_H] = 1
    return m


def adamw_step(p, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-4, decay=None):
    """One FP64 AdamW step on flat float64 arrays p, m, v (updated in
    place) with gradient g; step counts from 1."""
    lib = _load()
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, np.float64)
    dm = np.ascontiguousarray(decay_mask() if decay is None else decay, np.uint8)
    assert len(p) == len(m) == len(v) == len(g) == len(dm)
    lib.ora_adamw_step(len(p), _p(p), _p(m), _p(v), _p(g), _p(dm), float(lr), float(beta1), float(beta2),
                       float(eps), float(weight_decay), int(step))
    return p


def mlp_features(yd, td, xd, yi, ti, xi, yu, tu, xu, g, wy, wt, w, c2s, n_cand):
    lib = _load()
    f = np.zeros(MLP_INP, np.float32)
    lib.ora_mlp_features(yd, td, xd, yi, ti, xi, yu, tu, xu, g, wy, wt, w, c2s, n_cand, _p(f))
    return f


def triplets(cfg: Config, row, y, t, cap=None):
    """Every accepted triplet (d, i, u, g) of a sector and its features."""
    lib = _load()
    row, y, t = _in(row, y, t)
    c = cfg._c()
    n = lib.ora_triplets(ctypes.byref(c), len(row), _p(row), _p(y), _p(t), 0, None, None)
    cap = n if cap is None else min(cap, n)
    tri = np.zeros((max(cap, 1), 4), np.int32)
    feat = np.zeros((max(cap, 1), MLP_INP), np.float32)
    lib.ora_triplets(ctypes.byref(c), len(row), _p(row), _p(y), _p(t), cap, _p(tri), _p(feat))
    return tri[:cap], feat[:cap]


def links_pruned(cfg: Config, row, y, t, m: MLP, theta: float, tol: float = 1e-3):
    """Links with the triplet network gate (logit >= theta); near[i] counts
    hit i's triplets within tol of theta."""
    lib = _load()
    row, y, t = _in(row, y, t)
    n = len(row)
    up = np.empty(n, np.int32); dn = np.empty(n, np.int32); gap = np.empty(n, np.int32)
    near = np.zeros(n, np.int32)
    w = m.flat()
    c = cfg._c()
    lib.ora_links_pruned(ctypes.byref(c), n, _p(row), _p(y), _p(t), _p(w), float(theta), float(tol),
                         _p(up), _p(dn), _p(gap), _p(near))
    return up, dn, gap, near
