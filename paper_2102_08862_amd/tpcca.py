"""Python binding of libtpcca.so (the MI355X TPC track finder).

Argument marshalling only: every step of the tracking runs in the library's
HIP kernels. PyTorch provides the device memory (the arena and, optionally,
device-resident inputs) and the stream. There is no CPU fallback: if the
library is not built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpcca.so")
HEADER = os.path.join(_HERE, "..", "include", "tpcca.h")

OK, ERR_INVALID_ARG, ERR_NOMEM, ERR_CAPACITY, ERR_STATE, ERR_DEVICE, ERR_ABORTED = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "NOMEM", -3: "CAPACITY", -4: "STATE", -5: "DEVICE", -6: "ABORTED"}


class TpccaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("tpcca %s: %s" % (_NAMES.get(status, status), msg))
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("bz_tesla", ctypes.c_float),
        ("n_sectors", ctypes.c_int32),
        ("n_rows", ctypes.c_int32),
        ("row_x", ctypes.POINTER(ctypes.c_float)),
        ("sigma_y", ctypes.c_float), ("sigma_t", ctypes.c_float),
        ("win_y", ctypes.c_float), ("win_t", ctypes.c_float),
        ("pair_c2", ctypes.c_float),
        ("max_gap", ctypes.c_int32),
        ("min_track_hits", ctypes.c_int32),
        ("prior_var_sinphi", ctypes.c_float),
        ("prior_var_tau", ctypes.c_float),
        ("prior_var_qpt", ctypes.c_float),
        ("kf_passes", ctypes.c_int32),
        ("s_max", ctypes.c_float),
        ("use_mlp", ctypes.c_int32),
        ("mlp_logit_threshold", ctypes.c_float),
        ("pool_per_cluster", ctypes.c_int32),
        ("follow", ctypes.c_int32),
        ("follow_win_y", ctypes.c_float), ("follow_win_t", ctypes.c_float),
        ("follow_chi2", ctypes.c_float), ("follow_q", ctypes.c_float),
        ("follow_var_y", ctypes.c_float), ("follow_var_t", ctypes.c_float),
        ("follow_var_slope0", ctypes.c_float),
        ("follow_max_miss", ctypes.c_int32),
    ]


TRACK_DTYPE = np.dtype([
    ("frame", np.int32), ("sector", np.int32), ("n_clusters", np.int32), ("status", np.int32),
    ("first", np.int64), ("seed", np.int32), ("ndf", np.int32),
    ("x_ref", np.float32), ("y", np.float32), ("t_base", np.float32), ("dt", np.float32),
    ("sinphi", np.float32), ("tau", np.float32), ("qpt", np.float32), ("chi2", np.float32),
    ("cov", np.float32, (15,)),
], align=True)


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_clusters", ctypes.c_int64), ("n_links", ctypes.c_int64), ("n_seeds", ctypes.c_int64),
        ("n_tracks", ctypes.c_int64), ("n_track_clusters", ctypes.c_int64), ("n_invalid", ctypes.c_int64),
        ("n_overflow_tiles", ctypes.c_int64), ("n_triplets", ctypes.c_int64), ("n_pruned", ctypes.c_int64),
        ("n_pool_overflow", ctypes.c_int64), ("mlp_used", ctypes.c_int32),
        ("n_timed_runs", ctypes.c_int64),
        ("n_stages", ctypes.c_int32),
        ("stage_ms", ctypes.c_float * 16),
        ("stage_ms_total", ctypes.c_double * 16),
        ("stage_name", (ctypes.c_char * 24) * 16),
        ("n_tiles", ctypes.c_int64), ("fit_passes", ctypes.c_int64 * 16), ("n_fit_restarts", ctypes.c_int64),
        ("n_chains", ctypes.c_int64), ("n_follow_added", ctypes.c_int64), ("n_follow_dropped", ctypes.c_int64),
    ]


# every entry point declared in include/tpcca.h
EXPORTS = [
    "tpcca_config_default", "tpcca_create", "tpcca_destroy", "tpcca_last_error", "tpcca_set_stream",
    "tpcca_add_frame", "tpcca_clear_frames", "tpcca_load_sector", "tpcca_required_arena",
    "tpcca_attach_arena", "tpcca_run", "tpcca_run_noalloc", "tpcca_synchronize", "tpcca_request_abort", "tpcca_set_timing",
    "tpcca_get_stats", "tpcca_get_tracks", "tpcca_get_track_clusters", "tpcca_get_assignment",
    "tpcca_get_links", "tpcca_mlp_state_bytes", "tpcca_mlp_attach", "tpcca_mlp_load", "tpcca_mlp_fetch",
    "tpcca_mlp_infer", "tpcca_mlp_grad", "tpcca_mlp_train_step", "tpcca_get_triplets", "tpcca_set_graph",
    "tpcca_set_launch", "tpcca_set_pruning", "tpcca_set_triplet_pool", "tpcca_copy", "tpcca_triplet_samples",
    "tpcca_find_collisions", "tpcca_get_track_times", "tpcca_get_collisions", "tpcca_merge_sectors",
    "tpcca_get_merges", "tpcca_refit_merged", "tpcca_get_refits", "tpcca_merge_membrane",
    "tpcca_get_membrane_merges", "tpcca_remove_clusters", "tpcca_get_removal_range", "tpcca_entropy_histograms",
    "tpcca_ans_encode",
]

MLP_NPARAM = 5313


class MlpHparams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("weight_decay", ctypes.c_float), ("pos_weight", ctypes.c_float)]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtpcca.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libtpcca.so is not built (run __graft_entry__.build() or "
                           "python paper_2102_08862_amd/build.py)")
    lib = ctypes.CDLL(path)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "tpcca_config_default": [ctypes.POINTER(Config)],
        "tpcca_create": [ctypes.POINTER(Config), ctypes.POINTER(P)],
        "tpcca_set_stream": [P, P],
        "tpcca_add_frame": [P, ctypes.POINTER(I32)],
        "tpcca_clear_frames": [P],
        "tpcca_load_sector": [P, I32, I32, I64, P, P, P, I32],
        "tpcca_required_arena": [P, ctypes.POINTER(SZ)],
        "tpcca_attach_arena": [P, P, SZ],
        "tpcca_run": [P],
        "tpcca_run_noalloc": [P],
        "tpcca_synchronize": [P],
        "tpcca_request_abort": [P],
        "tpcca_set_timing": [P, I32],
        "tpcca_get_stats": [P, ctypes.POINTER(Stats)],
        "tpcca_get_tracks": [P, I32, I32, P, I64, ctypes.POINTER(I64)],
        "tpcca_get_track_clusters": [P, I32, I32, P, I64, ctypes.POINTER(I64)],
        "tpcca_get_assignment": [P, I32, I32, P, I64],
        "tpcca_find_collisions": [P, ctypes.c_float, I32, ctypes.c_float, ctypes.POINTER(I64)],
        "tpcca_get_track_times": [P, I32, I32, P, P, I64, ctypes.POINTER(I64)],
        "tpcca_get_collisions": [P, I32, I32, P, P, P, I64, ctypes.POINTER(I64)],
        "tpcca_merge_sectors": [P, I32, ctypes.c_float, ctypes.c_float, ctypes.POINTER(I64)],
        "tpcca_get_merges": [P, I32, I32, P, P, I64, ctypes.POINTER(I64)],
        "tpcca_refit_merged": [P, ctypes.POINTER(I64)],
        "tpcca_merge_membrane": [P, I32, ctypes.c_float, ctypes.c_float, ctypes.POINTER(I64)],
        "tpcca_get_membrane_merges": [P, I32, I32, P, I64, ctypes.POINTER(I64)],
        "tpcca_remove_clusters": [P, ctypes.c_float, P, I64, ctypes.POINTER(I64)],
        "tpcca_get_removal_range": [P, I32, I32, ctypes.POINTER(I64), ctypes.POINTER(I64)],
        "tpcca_entropy_histograms": [P, I32, I32, P],
        "tpcca_ans_encode": [P, I32, I32, P, I64, P, I64, ctypes.POINTER(I64)],
        "tpcca_get_refits": [P, I32, I32, P, P, P, I64, ctypes.POINTER(I64)],
        "tpcca_get_links": [P, I32, I32, I32, P, P, I64],
        "tpcca_mlp_state_bytes": [ctypes.POINTER(SZ)],
        "tpcca_mlp_attach": [P, P, SZ],
        "tpcca_mlp_load": [P, P],
        "tpcca_mlp_fetch": [P, P],
        "tpcca_mlp_infer": [P, P, I64, P],
        "tpcca_mlp_grad": [P, P, P, I64, ctypes.c_float, P, P],
        "tpcca_mlp_train_step": [P, P, P, I64, ctypes.POINTER(MlpHparams), P],
        "tpcca_get_triplets": [P, I32, I32, P, P, P, I64, ctypes.POINTER(I64)],
        "tpcca_set_graph": [P, I32],
        "tpcca_set_launch": [P, I32, I32, I32],
        "tpcca_set_pruning": [P, I32, ctypes.c_float],
        "tpcca_set_triplet_pool": [P, I32],
        "tpcca_copy": [P, P, P, SZ],
        "tpcca_triplet_samples": [P, ctypes.c_float, ctypes.c_uint64, P, P, I64, ctypes.POINTER(I64)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.tpcca_destroy.argtypes = [P]
    lib.tpcca_destroy.restype = None
    lib.tpcca_last_error.argtypes = [P]
    lib.tpcca_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def default_config() -> Config:
    lib = load_library()
    c = Config()
    lib.tpcca_config_default(ctypes.byref(c))
    return c


class Tracker:
    """One tracking context on the current GPU (torch's current device)."""

    def __init__(self, config: Config | None = None, **overrides):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the TPC tracker needs a GPU (no CPU fallback)")
        self._torch = torch
        self.lib = load_library()
        cfg = config if config is not None else default_config()
        self._row_x_keep = None
        for k, v in overrides.items():
            if k == "row_x":
                arr = np.ascontiguousarray(v, np.float32)
                self._row_x_keep = arr
                cfg.row_x = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
                cfg.n_rows = len(arr)
            else:
                setattr(cfg, k, v)
        self.config = cfg
        h = ctypes.c_void_p()
        self._check(self.lib.tpcca_create(ctypes.byref(cfg), ctypes.byref(h)), None)
        self.h = h
        self.arena = None
        self._keep = []          # device inputs borrowed by the library
        self.n_frames = 0
        self.sector_n = {}
        self.set_stream(torch.cuda.current_stream())

    # ------------------------------------------------------------ helpers
    def _check(self, st, h=-1):
        if st != OK:
            hh = self.h if h == -1 else h
            msg = self.lib.tpcca_last_error(hh).decode() if hh else ""
            raise TpccaError(st, msg)

    def _check_cap(self, st):
        """A size query: CAPACITY (the buffer of 0 entries is too small) is expected."""
        if st != OK and st != ERR_CAPACITY:
            self._check(st)

    def close(self):
        if getattr(self, "h", None):
            self.lib.tpcca_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        self._check(self.lib.tpcca_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)))

    # ------------------------------------------------------------- inputs
    def add_frame(self) -> int:
        f = ctypes.c_int32()
        self._check(self.lib.tpcca_add_frame(self.h, ctypes.byref(f)))
        self.n_frames = f.value + 1
        return f.value

    def clear_frames(self):
        self._check(self.lib.tpcca_clear_frames(self.h))
        self._keep = []
        self.sector_n = {}
        self.n_frames = 0

    def load_sector(self, frame, sector, row, y, t, device: bool = True):
        """Give one sector's clusters. numpy arrays (host, copied) or torch
        device tensors (borrowed); with device=True numpy inputs are first
        moved to device tensors that this object keeps alive."""
        torch = self._torch
        n = len(row)
        if isinstance(row, torch.Tensor):
            tr, ty, tt = row, y, t
            assert tr.is_cuda and tr.dtype == torch.uint8 and ty.dtype == torch.float32 and tt.dtype == torch.float32
            assert tr.is_contiguous() and ty.is_contiguous() and tt.is_contiguous()
            self._keep += [tr, ty, tt]
            ptrs = (tr.data_ptr(), ty.data_ptr(), tt.data_ptr())
            is_dev = 1
        elif device:
            tr = torch.from_numpy(np.ascontiguousarray(row, np.uint8)).cuda()
            ty = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
            tt = torch.from_numpy(np.ascontiguousarray(t, np.float32)).cuda()
            torch.cuda.synchronize()
            self._keep += [tr, ty, tt]
            ptrs = (tr.data_ptr(), ty.data_ptr(), tt.data_ptr())
            is_dev = 1
        else:
            r = np.ascontiguousarray(row, np.uint8)
            yy = np.ascontiguousarray(y, np.float32)
            ttt = np.ascontiguousarray(t, np.float32)
            ptrs = (r.ctypes.data, yy.ctypes.data, ttt.ctypes.data)
            is_dev = 0
        if n == 0:
            ptrs = (None, None, None)
        self._check(self.lib.tpcca_load_sector(self.h, frame, sector, n, ptrs[0], ptrs[1], ptrs[2], is_dev))
        self.sector_n[(frame, sector)] = n

    def load_frame(self, fr, frame=None, device: bool = True, sectors=None):
        """Load every sector of a generated frame (paper_2102_08862_amd.synth.Frame)."""
        if frame is None:
            frame = self.add_frame()
        ss = range(len(fr.rows)) if sectors is None else sectors
        for s in ss:
            self.load_sector(frame, s, fr.rows[s], fr.ys[s], fr.ts[s], device=device)
        return frame

    def load_frame_packed(self, fr, frame=None):
        """Copy a whole frame into three device tensors (one H2D each) and
        load every sector as a borrowed slice of them."""
        torch = self._torch
        if frame is None:
            frame = self.add_frame()
        ns = [len(r) for r in fr.rows]
        off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
        row = torch.from_numpy(np.concatenate(fr.rows) if off[-1] else np.zeros(0, np.uint8)).cuda()
        y = torch.from_numpy(np.concatenate(fr.ys) if off[-1] else np.zeros(0, np.float32)).cuda()
        t = torch.from_numpy(np.concatenate(fr.ts) if off[-1] else np.zeros(0, np.float32)).cuda()
        torch.cuda.synchronize()
        for s, n in enumerate(ns):
            a, b = int(off[s]), int(off[s + 1])
            self.load_sector(frame, s, row[a:b], y[a:b], t[a:b])
        return frame

    # ---------------------------------------------------------------- run
    def required_arena(self) -> int:
        b = ctypes.c_size_t()
        self._check(self.lib.tpcca_required_arena(self.h, ctypes.byref(b)))
        return b.value

    def ensure_arena(self):
        need = self.required_arena()
        if self.arena is None or self.arena.numel() < need:
            self.arena = None
            self.arena = self._torch.empty(need + 4096, dtype=self._torch.uint8, device="cuda")
            base = self.arena.data_ptr()
            aligned = (base + 255) // 256 * 256
            self._check(self.lib.tpcca_attach_arena(self.h, ctypes.c_void_p(aligned), need))
        return need

    def use_arena(self, buf):
        """Attach a caller-provided device buffer (torch uint8 tensor) as the
        arena, e.g. one buffer shared by several trackers whose runs are
        serialised on one stream."""
        need = self.required_arena()
        base = buf.data_ptr()
        aligned = (base + 255) // 256 * 256
        if buf.numel() - (aligned - base) < need:
            raise ValueError("arena buffer of %d bytes, run needs %d" % (buf.numel(), need))
        self.arena = buf
        self._check(self.lib.tpcca_attach_arena(self.h, ctypes.c_void_p(aligned), buf.numel() - (aligned - base)))
        return need

    def run(self, sync: bool = False):
        self.ensure_arena()
        self._check(self.lib.tpcca_run(self.h))
        if sync:
            self.synchronize()

    def run_noalloc(self, sync: bool = False):
        """Run with the library's static device arena (no arena, no allocation)."""
        self._check(self.lib.tpcca_run_noalloc(self.h))
        if sync:
            self.synchronize()

    def synchronize(self):
        self._check(self.lib.tpcca_synchronize(self.h))

    def request_abort(self):
        self._check(self.lib.tpcca_request_abort(self.h))

    def set_graph(self, on: bool):
        """Replay runs from a captured HIP graph (needs a non-default stream)."""
        if on and self.stream.cuda_stream == 0:
            self.set_stream(self._torch.cuda.Stream())
        self._check(self.lib.tpcca_set_graph(self.h, 1 if on else 0))

    def set_launch(self, stage: int, blocks_per_cu: int = 0, param: int = 0):
        self._check(self.lib.tpcca_set_launch(self.h, stage, blocks_per_cu, param))

    def set_pruning(self, use_mlp: bool, threshold: float = 0.0):
        """Switch triplet pruning on or off and set the logit threshold."""
        self._check(self.lib.tpcca_set_pruning(self.h, 1 if use_mlp else 0, float(threshold)))
        self.config.use_mlp = 1 if use_mlp else 0
        self.config.mlp_logit_threshold = float(threshold)

    def set_triplet_pool(self, keep: bool):
        """Pruned runs list every triplet in a pool (for triplets() and
        triplet_samples()) instead of scoring them inside the search."""
        self._check(self.lib.tpcca_set_triplet_pool(self.h, 1 if keep else 0))

    def copy(self, src, dst):
        """Plain device copy kernel (counter calibration): src -> dst, torch tensors."""
        n = src.numel() * src.element_size()
        assert dst.numel() * dst.element_size() >= n
        self._check(self.lib.tpcca_copy(self.h, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n))

    def set_timing(self, on: bool):
        self._check(self.lib.tpcca_set_timing(self.h, 1 if on else 0))

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.tpcca_get_stats(self.h, ctypes.byref(s)))
        d = {k: getattr(s, k) for k in ("n_clusters", "n_links", "n_seeds", "n_tracks", "n_track_clusters",
                                        "n_invalid", "n_overflow_tiles", "n_triplets", "n_pruned",
                                        "n_pool_overflow", "mlp_used", "n_tiles", "n_chains", "n_follow_added",
                                        "n_follow_dropped")}
        d["stage_ms"] = {s.stage_name[i].value.decode(): s.stage_ms[i] for i in range(s.n_stages)}
        d["fit_passes"] = [int(v) for v in s.fit_passes]
        d["n_fit_restarts"] = int(s.n_fit_restarts)
        d["n_timed_runs"] = s.n_timed_runs
        d["stage_ms_total"] = {s.stage_name[i].value.decode(): s.stage_ms_total[i] for i in range(s.n_stages)}
        return d

    # ------------------------------------------------------------ outputs
    def tracks(self, frame, sector) -> np.ndarray:
        n = ctypes.c_int64()
        st = self.lib.tpcca_get_tracks(self.h, frame, sector, None, 0, ctypes.byref(n))
        if st not in (OK, ERR_CAPACITY):
            self._check(st)
        out = np.zeros(n.value, TRACK_DTYPE)
        if n.value:
            self._check(self.lib.tpcca_get_tracks(self.h, frame, sector, out.ctypes.data, n.value, ctypes.byref(n)))
        return out

    def track_clusters(self, frame, sector) -> np.ndarray:
        n = ctypes.c_int64()
        st = self.lib.tpcca_get_track_clusters(self.h, frame, sector, None, 0, ctypes.byref(n))
        if st not in (OK, ERR_CAPACITY):
            self._check(st)
        out = np.zeros(n.value, np.int32)
        if n.value:
            self._check(self.lib.tpcca_get_track_clusters(self.h, frame, sector, out.ctypes.data, n.value,
                                                          ctypes.byref(n)))
        return out

    def assignment(self, frame, sector) -> np.ndarray:
        n = self.sector_n.get((frame, sector), 0)
        out = np.zeros(n, np.int32)
        self._check(self.lib.tpcca_get_assignment(self.h, frame, sector, out.ctypes.data if n else None, n))
        return out

    def find_collisions(self, gap_cm: float = 0.5, min_clusters: int = 60, window_cm: float = 5.0) -> int:
        """Group the tracks of every loaded frame side into collision
        candidates by their collision times: tracks of at least min_clusters
        clusters form the groups (a new one where t0 jumps by more than
        gap_cm), the others join the nearest group time within window_cm.
        Returns the number of groups."""
        n = ctypes.c_int64()
        self._check(self.lib.tpcca_find_collisions(self.h, float(gap_cm), int(min_clusters), float(window_cm),
                                                   ctypes.byref(n)))
        return n.value

    def track_times(self, frame, sector):
        """(t0 float32, group int32) of every track of the sector."""
        n = ctypes.c_int64()
        self._check_cap(self.lib.tpcca_get_track_times(self.h, frame, sector, None, None, 0, ctypes.byref(n)))
        t0 = np.zeros(n.value, np.float32)
        g = np.zeros(n.value, np.int32)
        if n.value:
            self._check(self.lib.tpcca_get_track_times(self.h, frame, sector, t0.ctypes.data, g.ctypes.data, n.value,
                                                       ctypes.byref(n)))
        return t0, g

    def collisions(self, frame, side):
        """(time float32, tracks int32, anchors int32) of every group of a
        frame side (0: A, 1: C), in ascending time."""
        n = ctypes.c_int64()
        self._check_cap(self.lib.tpcca_get_collisions(self.h, frame, side, None, None, None, 0, ctypes.byref(n)))
        t0 = np.zeros(n.value, np.float32)
        cnt = np.zeros(n.value, np.int32)
        anc = np.zeros(n.value, np.int32)
        if n.value:
            self._check(self.lib.tpcca_get_collisions(self.h, frame, side, t0.ctypes.data, cnt.ctypes.data,
                                                      anc.ctypes.data, n.value, ctypes.byref(n)))
        return t0, cnt, anc

    def merge_sectors(self, min_clusters: int = 30, window_cm: float = 8.0, d2_cut: float = 25.0) -> int:
        """Pair the tracks that continue each other across the border of two
        adjacent sectors of one side; returns the number of merged pairs."""
        n = ctypes.c_int64()
        self._check(self.lib.tpcca_merge_sectors(self.h, int(min_clusters), float(window_cm), float(d2_cut),
                                                 ctypes.byref(n)))
        return n.value

    def merges(self, frame, sector):
        """(next int32, prev int32): per track of the sector, the index of its
        merged partner among the next / previous sector's tracks (-1: none)."""
        n = ctypes.c_int64()
        self._check_cap(self.lib.tpcca_get_merges(self.h, frame, sector, None, None, 0, ctypes.byref(n)))
        nx = np.full(n.value, -1, np.int32)
        pv = np.full(n.value, -1, np.int32)
        if n.value:
            self._check(self.lib.tpcca_get_merges(self.h, frame, sector, nx.ctypes.data, pv.ctypes.data, n.value,
                                                  ctypes.byref(n)))
        return nx, pv

    def merge_membrane(self, min_clusters: int = 30, window_cm: float = 30.0, d2_cut: float = 25.0) -> int:
        """Pair the tracks of one particle on the two sides of the central
        membrane (sector k and k + 18); returns the number of merged pairs."""
        n = ctypes.c_int64()
        self._check(self.lib.tpcca_merge_membrane(self.h, int(min_clusters), float(window_cm), float(d2_cut),
                                                  ctypes.byref(n)))
        return n.value

    def membrane_merges(self, frame, sector):
        """int32 per track of the sector: its membrane partner's index among
        the other side's sector's tracks (-1: none)."""
        n = ctypes.c_int64()
        self._check_cap(self.lib.tpcca_get_membrane_merges(self.h, frame, sector, None, 0, ctypes.byref(n)))
        out = np.full(n.value, -1, np.int32)
        if n.value:
            self._check(self.lib.tpcca_get_membrane_merges(self.h, frame, sector, out.ctypes.data, n.value,
                                                           ctypes.byref(n)))
        return out

    def remove_clusters(self, pt_min: float = 0.15):
        """Drop the clusters of fitted tracks below pt_min (GeV): returns a
        device int32 tensor of the kept clusters' input indices, sector
        after sector (removal_range gives each sector's part)."""
        import torch
        n = ctypes.c_int64()
        self._check_cap(self.lib.tpcca_remove_clusters(self.h, float(pt_min), None, 0, ctypes.byref(n)))
        out = torch.empty(max(n.value, 1), dtype=torch.int32, device="cuda")
        self._check(self.lib.tpcca_remove_clusters(self.h, float(pt_min), ctypes.c_void_p(out.data_ptr()), n.value,
                                                   ctypes.byref(n)))
        return out[:n.value]

    def removal_range(self, frame, sector):
        """(begin, count) of the sector's kept clusters in remove_clusters' output."""
        b, c = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.tpcca_get_removal_range(self.h, frame, sector, ctypes.byref(b), ctypes.byref(c)))
        return b.value, c.value

    def entropy_histograms(self, frame: int = -1, sector: int = -1) -> np.ndarray:
        """int64 [5, 512] symbol histograms of the track clusters (row step;
        y, t first differences; y, t track-model residuals) of the run, or of
        one sector."""
        h = np.zeros((5, 512), np.int64)
        self._check(self.lib.tpcca_entropy_histograms(self.h, int(frame), int(sector), h.ctypes.data))
        return h

    def ans_encode(self, frame, sector):
        """rANS bytes of the sector's track clusters: (device uint8 tensor,
        int64 offsets of every track's bytes, then the end)."""
        import torch
        n = ctypes.c_int64()
        self._check_cap(self.lib.tpcca_ans_encode(self.h, frame, sector, None, 0, None, 0, ctypes.byref(n)))
        nt = len(self.tracks(frame, sector))
        out = torch.empty(max(n.value, 1), dtype=torch.uint8, device="cuda")
        off = np.zeros(nt + 1, np.int64)
        self._check(self.lib.tpcca_ans_encode(self.h, frame, sector, ctypes.c_void_p(out.data_ptr()), n.value,
                                              off.ctypes.data, len(off), ctypes.byref(n)))
        return out[:n.value], off

    def refit_merged(self) -> int:
        """Fit every merged pair as one track (clusters of both in the first
        track's sector frame); returns the number of pairs refitted."""
        n = ctypes.c_int64()
        self._check(self.lib.tpcca_refit_merged(self.h, ctypes.byref(n)))
        return n.value

    def refits(self, frame, sector):
        """(tracks TRACK_DTYPE, first int32, partner int32): the refits whose
        first track lies in the sector, that track's index among the
        sector's tracks and its partner's among the next sector's."""
        n = ctypes.c_int64()
        self._check_cap(self.lib.tpcca_get_refits(self.h, frame, sector, None, None, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, TRACK_DTYPE)
        fi = np.full(n.value, -1, np.int32)
        pa = np.full(n.value, -1, np.int32)
        if n.value:
            self._check(self.lib.tpcca_get_refits(self.h, frame, sector, out.ctypes.data, fi.ctypes.data,
                                                  pa.ctypes.data, n.value, ctypes.byref(n)))
        return out, fi, pa

    def links(self, frame, sector, cleaned: bool = False):
        n = self.sector_n.get((frame, sector), 0)
        up = np.zeros(n, np.int32)
        dn = np.zeros(n, np.int32)
        self._check(self.lib.tpcca_get_links(self.h, frame, sector, 1 if cleaned else 0,
                                             up.ctypes.data if n else None, dn.ctypes.data if n else None, n))
        return up, dn

    # ------------------------------------------------------ triplet network
    def mlp_attach(self):
        torch = self._torch
        b = ctypes.c_size_t()
        self._check(self.lib.tpcca_mlp_state_bytes(ctypes.byref(b)))
        self.mlp_state = torch.zeros(b.value + 256, dtype=torch.uint8, device="cuda")
        base = (self.mlp_state.data_ptr() + 255) // 256 * 256
        self._check(self.lib.tpcca_mlp_attach(self.h, ctypes.c_void_p(base), b.value))

    def mlp_load(self, params):
        """params: 5313 FP32 values (w1[64][16], b1, w2[64][64], b2, w3, b3)."""
        if getattr(self, "mlp_state", None) is None:
            self.mlp_attach()
        p = np.ascontiguousarray(params, np.float32)
        assert p.size == MLP_NPARAM
        self._check(self.lib.tpcca_mlp_load(self.h, p.ctypes.data))

    def mlp_fetch(self):
        p = np.zeros(MLP_NPARAM, np.float32)
        self._check(self.lib.tpcca_mlp_fetch(self.h, p.ctypes.data))
        return p

    def mlp_infer(self, x_dev, z_dev=None):
        """x_dev: torch int16/uint16-bit tensor [n, 16] of BF16 features on the GPU."""
        n = x_dev.shape[0]
        if z_dev is None:
            z_dev = self._torch.empty(n, dtype=self._torch.float32, device="cuda")
        self._check(self.lib.tpcca_mlp_infer(self.h, ctypes.c_void_p(x_dev.data_ptr()), n,
                                             ctypes.c_void_p(z_dev.data_ptr())))
        return z_dev

    def mlp_grad(self, x_dev, y_dev, pos_weight=1.0):
        torch = self._torch
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        self._check(self.lib.tpcca_mlp_grad(self.h, ctypes.c_void_p(x_dev.data_ptr()),
                                            ctypes.c_void_p(y_dev.data_ptr()), x_dev.shape[0], float(pos_weight),
                                            ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(loss.data_ptr())))
        return g, loss

    def mlp_train_step(self, x_dev, y_dev, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-4,
                       pos_weight=1.0, loss_dev=None):
        hp = MlpHparams(lr, beta1, beta2, eps, weight_decay, pos_weight)
        self._check(self.lib.tpcca_mlp_train_step(self.h, ctypes.c_void_p(x_dev.data_ptr()),
                                                  ctypes.c_void_p(y_dev.data_ptr()), x_dev.shape[0], ctypes.byref(hp),
                                                  ctypes.c_void_p(loss_dev.data_ptr()) if loss_dev is not None else None))

    def triplet_samples(self, keep: float, seed: int, cap: int):
        """Labelled training triplets of the last pruned run, on the device:
        (feat int16 [n, 16] BF16 bits, label float32 [n])."""
        torch = self._torch
        feat = torch.empty((max(cap, 1), 16), dtype=torch.int16, device="cuda")
        lab = torch.empty(max(cap, 1), dtype=torch.float32, device="cuda")
        n = ctypes.c_int64()
        self._check(self.lib.tpcca_triplet_samples(self.h, float(keep), int(seed) & 0xffffffffffffffff,
                                                   ctypes.c_void_p(feat.data_ptr()), ctypes.c_void_p(lab.data_ptr()),
                                                   cap, ctypes.byref(n)))
        return feat[:n.value], lab[:n.value]

    def triplets(self, frame, sector):
        """(tri int32[n,4] = (down, cluster, up, gap) input ids, feat uint16[n,16], z float32[n])."""
        n = ctypes.c_int64()
        st = self.lib.tpcca_get_triplets(self.h, frame, sector, None, None, None, 0, ctypes.byref(n))
        if st not in (OK, ERR_CAPACITY):
            self._check(st)
        tri = np.zeros((n.value, 4), np.int32)
        feat = np.zeros((n.value, 16), np.uint16)
        z = np.zeros(n.value, np.float32)
        if n.value:
            self._check(self.lib.tpcca_get_triplets(self.h, frame, sector, tri.ctypes.data, feat.ctypes.data,
                                                    z.ctypes.data, n.value, ctypes.byref(n)))
        return tri, feat, z
