"""Seeded synthetic TPC time frames (input generator shared by the tracker's
tests, its benchmark and the CPU oracle's tests).

It simulates helices from Pb-Pb-like collisions and records one cluster
(pad row, y, drift time) per crossed pad row, in the native TPC coordinates
the paper says the tracking must work in (Sec. 1: hits stay in time / pad-row
/ pad coordinates because collisions are not known before tracking). It holds
no part of the tracking method itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libtpcsynth.so")

N_ROWS = 152
N_SECTORS = 36


class _Params(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("single_sector", ctypes.c_int32),
        ("n_collisions", ctypes.c_int32),
        ("fixed_mult", ctypes.c_int32),
        ("frame_us", ctypes.c_double),
        ("bz", ctypes.c_double),
        ("sigma_y", ctypes.c_double),
        ("sigma_t", ctypes.c_double),
        ("noise_frac", ctypes.c_double),
        ("quant", ctypes.c_double),
        ("mult_mean", ctypes.c_double),
        ("mult_max", ctypes.c_double),
        ("pt_min", ctypes.c_double),
        ("pt_mean", ctypes.c_double),
        ("eta_max", ctypes.c_double),
        ("zv_sigma", ctypes.c_double),
        ("vdrift", ctypes.c_double),
        ("drift_len", ctypes.c_double),
        ("n_threads", ctypes.c_int32),
    ]


def build(force: bool = False) -> str:
    """Compile the generator with gcc (plain C, pthreads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.synth_generate.restype = ctypes.c_void_p
        lib.synth_generate.argtypes = [ctypes.POINTER(_Params)]
        lib.synth_params_default.argtypes = [ctypes.POINTER(_Params)]
        lib.synth_sector_count.restype = ctypes.c_int64
        lib.synth_sector_count.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        lib.synth_sector_copy.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 4
        lib.synth_n_tracks.restype = ctypes.c_int64
        lib.synth_n_tracks.argtypes = [ctypes.c_void_p]
        lib.synth_tracks_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_time_range.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
        lib.synth_free.argtypes = [ctypes.c_void_p]
        lib.synth_geometry.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_helix_at.restype = ctypes.c_int32
        lib.synth_helix_at.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        _lib = lib
    return _lib


def geometry(n_rows: int = N_ROWS):
    """Pad-row positions x_r (cm) and half widths (cm), float32."""
    lib = _load()
    x = np.zeros(n_rows, np.float32)
    hw = np.zeros(n_rows, np.float32)
    lib.synth_geometry(n_rows, x.ctypes.data, hw.ctypes.data)
    return x, hw


# Workloads named by what they are (all at 50 kHz Pb-Pb, 0.5 T, sigma 0.1 cm, 5% noise).
WORKLOADS = {
    # one sector, 300 primary helices from one vertex, t = z
    "sector_300": dict(single_sector=1, n_collisions=1, fixed_mult=300, frame_us=0.0),
    # all 36 sectors, 1 ms continuous slice, 50 collisions
    "slice_1ms": dict(n_collisions=50, frame_us=1000.0),
    # all 36 sectors, full 10 ms time frame, 500 collisions
    "frame_10ms": dict(n_collisions=500, frame_us=10000.0),
}


@dataclass
class Frame:
    seed: int
    params: dict
    rows: list = field(default_factory=list)     # per sector uint8[n]
    ys: list = field(default_factory=list)       # per sector float32[n]
    ts: list = field(default_factory=list)       # per sector float32[n]
    labels: list = field(default_factory=list)   # per sector int32[n] (track id, -1 noise)
    tracks: np.ndarray = None                    # [n_tracks, 8] q, pt, phi0, tgl, zv, tcoll_us, kappa, eta
    t_range: tuple = (0.0, 0.0)

    @property
    def n_clusters(self) -> int:
        return int(sum(len(r) for r in self.rows))

    def sector(self, s):
        return self.rows[s], self.ys[s], self.ts[s]


def generate(workload: str | None = None, seed: int = 1, n_threads: int | None = None, **overrides) -> Frame:
    """Generate one frame. `workload` picks a preset from WORKLOADS; keyword
    overrides set any generator parameter (sigma_y, noise_frac, quant, bz,
    n_collisions, frame_us, fixed_mult, single_sector, ...)."""
    lib = _load()
    p = _Params()
    lib.synth_params_default(ctypes.byref(p))
    kw = dict(WORKLOADS[workload]) if workload else {}
    kw.update(overrides)
    for k, v in kw.items():
        setattr(p, k, v)
    p.seed = seed
    p.n_threads = n_threads if n_threads else min(16, os.cpu_count() or 1)
    h = lib.synth_generate(ctypes.byref(p))
    try:
        fr = Frame(seed=seed, params={k: getattr(p, k) for k, _ in _Params._fields_})
        nsec = 1 if p.single_sector else N_SECTORS
        for s in range(nsec):
            n = lib.synth_sector_count(h, s)
            row = np.empty(n, np.uint8)
            y = np.empty(n, np.float32)
            t = np.empty(n, np.float32)
            lab = np.empty(n, np.int32)
            lib.synth_sector_copy(h, s, row.ctypes.data, y.ctypes.data, t.ctypes.data, lab.ctypes.data)
            fr.rows.append(row)
            fr.ys.append(y)
            fr.ts.append(t)
            fr.labels.append(lab)
        nt = lib.synth_n_tracks(h)
        tr = np.empty((nt, 8), np.float64)
        if nt:
            lib.synth_tracks_copy(h, tr.ctypes.data)
        fr.tracks = tr
        lo, hi = ctypes.c_double(), ctypes.c_double()
        lib.synth_time_range(h, ctypes.byref(lo), ctypes.byref(hi))
        fr.t_range = (lo.value, hi.value)
        return fr
    finally:
        lib.synth_free(h)


def helix_at(track8, sector: int, x: float, single_sector: bool, vdrift: float = 2.58, drift_len: float = 250.0):
    """Truth helix of a generated track at the row line X = x of a sector:
    returns (Y, z, sin(local phi), arc, t, dt/darc) or None if not crossed."""
    lib = _load()
    trk = np.ascontiguousarray(track8, np.float64)
    out = np.zeros(6, np.float64)
    ok = lib.synth_helix_at(trk.ctypes.data, sector, float(x), int(single_sector), vdrift, drift_len,
                            out.ctypes.data)
    return tuple(out) if ok else None
