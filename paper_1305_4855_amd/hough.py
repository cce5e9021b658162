"""Thin ctypes binding of libhough.so (include/hough.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Tensors are used for device memory and streams; the library is
loaded from this package directory and a missing library raises at import
(there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhough.so")

HOUGH_F_PEAK_OVERFLOW = 1
HOUGH_F_PAIR_OVERFLOW = 2


class HoughError(RuntimeError):
    pass


class Geometry(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("r_cm", C.POINTER(C.c_double)),
                ("halflen_cm", C.POINTER(C.c_double)), ("B_tesla", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("n_phi", C.c_int32), ("n_qpt", C.c_int32), ("n_d0", C.c_int32), ("frac_bits", C.c_int32),
                ("qpt_min", C.c_double), ("qpt_max", C.c_double), ("d0_min", C.c_double), ("d0_max", C.c_double),
                ("acc_bits", C.c_int32), ("n_cot", C.c_int32), ("n_z0", C.c_int32),
                ("cot_min", C.c_double), ("cot_max", C.c_double), ("z0_min", C.c_double), ("z0_max", C.c_double),
                ("max_hits_per_event", C.c_int32)]


class Hits(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("layer", C.c_void_p), ("n", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("vote_threads", C.c_int32), ("vote_grid", C.c_int32), ("peak_planes", C.c_int32),
                ("vote_cols", C.c_int32), ("assign_blocks", C.c_int32), ("prep_rows", C.c_int32)]


class VertexGrid(C.Structure):
    _fields_ = [("n_vr", C.c_int32), ("n_vphi", C.c_int32), ("r_min", C.c_double), ("r_max", C.c_double),
                ("min_votes", C.c_int32)]


class Batch(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("layer", C.c_void_p),
                ("hit_offsets", C.c_void_p), ("n_events", C.c_int32), ("threshold", C.c_int32),
                ("cap_peaks", C.c_int32), ("cap_pairs", C.c_int32), ("acc", C.c_void_p), ("peaks", C.c_void_p),
                ("offsets", C.c_void_p), ("hit_idx", C.c_void_p), ("ws", C.c_void_p), ("ws_bytes", C.c_size_t),
                ("status", C.c_void_p), ("zvote", C.c_void_p)]


STATUS_BYTES = 32
# workspace limit of hough_run_batch_noalloc (the library's per-GPU scratch array)
NOALLOC_SCRATCH_BYTES = 64 << 20
PEAK_INTS = 4
HOUGH_F_EVENT_TOO_LARGE = 4


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    P, S = C.c_void_p, C.c_size_t
    L.hough_plan_create.restype = C.c_int
    L.hough_plan_create.argtypes = [C.POINTER(Geometry), C.POINTER(Grid), C.POINTER(C.c_void_p)]
    L.hough_plan_destroy.restype = None; L.hough_plan_destroy.argtypes = [P]
    L.hough_acc_bytes.restype = S; L.hough_acc_bytes.argtypes = [P]
    L.hough_event_ws_bytes.restype = S; L.hough_event_ws_bytes.argtypes = [P, C.c_int32]
    L.hough_angle_bits.restype = C.c_int32; L.hough_angle_bits.argtypes = [P]
    L.hough_plan_table.restype = C.c_int; L.hough_plan_table.argtypes = [P, P]
    L.hough_prep.restype = C.c_int; L.hough_prep.argtypes = [P, C.POINTER(Hits), P, P, S, P, P]
    L.hough_vote.restype = C.c_int; L.hough_vote.argtypes = [P, C.POINTER(Hits), P, P, S, P, P]
    L.hough_vote_prepared.restype = C.c_int; L.hough_vote_prepared.argtypes = [P, P, P, S, P, P]
    L.hough_peaks.restype = C.c_int
    L.hough_peaks.argtypes = [P, P, C.c_int32, P, C.c_int32, P, S, P, P]
    L.hough_assign.restype = C.c_int
    L.hough_assign.argtypes = [P, P, C.c_int32, P, P, C.c_int32, P, S, P, P]
    L.hough_zvote.restype = C.c_int
    L.hough_zvote.argtypes = [P, C.POINTER(Hits), P, C.c_int32, P, P, C.c_int32, P, P, P]
    L.hough_fit.restype = C.c_int
    L.hough_fit.argtypes = [P, C.POINTER(Hits), P, P, C.c_int32, C.c_int32, P, P, P]
    L.hough_plan_arclen_table.restype = C.c_int; L.hough_plan_arclen_table.argtypes = [P, P]
    L.hough_strerror.restype = C.c_char_p; L.hough_strerror.argtypes = [C.c_int]
    L.hough_vote_cr.restype = C.c_int; L.hough_vote_cr.argtypes = [P, C.POINTER(Hits), P, P, P]
    L.hough_fit_batch.restype = C.c_int; L.hough_fit_batch.argtypes = [P, C.POINTER(Batch), P, P]
    L.hough_vertex_plan_create.restype = C.c_int
    L.hough_vertex_plan_create.argtypes = [P, C.POINTER(VertexGrid), C.POINTER(C.c_void_p)]
    L.hough_vertex_plan_destroy.restype = None; L.hough_vertex_plan_destroy.argtypes = [P]
    L.hough_vertex_set_groups.restype = C.c_int; L.hough_vertex_set_groups.argtypes = [P, C.c_int32]
    L.hough_vertex_get_groups.restype = C.c_int32; L.hough_vertex_get_groups.argtypes = [P]
    L.hough_vertex_vote_ws_bytes.restype = S; L.hough_vertex_vote_ws_bytes.argtypes = [P, C.c_int32]
    L.hough_vertex_peaks_ws_bytes.restype = S; L.hough_vertex_peaks_ws_bytes.argtypes = [P, C.c_int32]
    L.hough_vertex_vote.restype = C.c_int
    L.hough_vertex_vote.argtypes = [P, P, C.c_int32, P, P, P, S, P, P]
    L.hough_vertex_peaks.restype = C.c_int
    L.hough_vertex_peaks.argtypes = [P, P, C.c_int32, P, C.c_int32, P, S, P, P]
    L.hough_vertex_table.restype = C.c_int; L.hough_vertex_table.argtypes = [P, P]
    L.hough_vertex_batch_vote_ws_bytes.restype = S
    L.hough_vertex_batch_vote_ws_bytes.argtypes = [P, C.c_int32, C.c_int32]
    L.hough_vertex_batch_peaks_ws_bytes.restype = S
    L.hough_vertex_batch_peaks_ws_bytes.argtypes = [P, C.c_int32, C.c_int32]
    L.hough_vertex_vote_batch.restype = C.c_int
    L.hough_vertex_vote_batch.argtypes = [P, C.c_int32, P, C.c_int32, P, P, P, S, P, P]
    L.hough_vertex_peaks_batch.restype = C.c_int
    L.hough_vertex_peaks_batch.argtypes = [P, C.c_int32, P, C.c_int32, P, C.c_int32, P, S, P, P]
    L.hough_plan_set_tuning.restype = C.c_int; L.hough_plan_set_tuning.argtypes = [P, C.POINTER(Tuning)]
    L.hough_plan_get_tuning.restype = C.c_int; L.hough_plan_get_tuning.argtypes = [P, C.POINTER(Tuning)]
    L.hough_plan_set_vote_events.restype = C.c_int; L.hough_plan_set_vote_events.argtypes = [P, P, P]
    L.hough_plan_set_assign_events.restype = C.c_int; L.hough_plan_set_assign_events.argtypes = [P, P, P]
    L.hough_batch_ws_bytes.restype = S; L.hough_batch_ws_bytes.argtypes = [P, C.c_int32, C.c_int32]
    L.hough_run_batch.restype = C.c_int; L.hough_run_batch.argtypes = [P, C.POINTER(Batch), P]
    L.hough_run_batch_noalloc.restype = C.c_int; L.hough_run_batch_noalloc.argtypes = [P, C.POINTER(Batch), P]
    L.hough_refine.restype = C.c_int
    L.hough_refine.argtypes = [P, P, C.c_int32, P, P, C.c_int32, P, S, P, C.c_int32, P, P, P]
    L.hough_assign_cr_ws_bytes.restype = S; L.hough_assign_cr_ws_bytes.argtypes = [P, C.c_int32, C.c_int32]
    L.hough_assign_cr.restype = C.c_int
    L.hough_assign_cr.argtypes = [P, C.POINTER(Hits), P, C.c_int32, P, P, C.c_int32, P, S, P, S, P, P]
    L.hough_batch_graph_create.restype = C.c_int
    L.hough_batch_graph_create.argtypes = [P, C.POINTER(Batch), P, C.POINTER(C.c_void_p)]
    L.hough_graph_launch.restype = C.c_int; L.hough_graph_launch.argtypes = [P, P]
    L.hough_graph_destroy.restype = None; L.hough_graph_destroy.argtypes = [P]
    return L


lib = _load()

EXPORTED = ["hough_plan_create", "hough_plan_destroy", "hough_acc_bytes", "hough_event_ws_bytes",
            "hough_angle_bits", "hough_plan_table", "hough_prep", "hough_vote", "hough_vote_prepared", "hough_peaks",
            "hough_assign", "hough_zvote", "hough_fit", "hough_plan_arclen_table", "hough_strerror", "hough_plan_set_tuning", "hough_plan_get_tuning", "hough_plan_set_vote_events",
            "hough_plan_set_assign_events",
            "hough_batch_ws_bytes", "hough_run_batch", "hough_run_batch_noalloc", "hough_batch_graph_create",
            "hough_graph_launch",
            "hough_graph_destroy", "hough_fit_batch", "hough_vote_cr", "hough_assign_cr_ws_bytes", "hough_assign_cr", "hough_refine", "hough_vertex_plan_create", "hough_vertex_plan_destroy", "hough_vertex_set_groups",
            "hough_vertex_get_groups", "hough_vertex_vote_ws_bytes", "hough_vertex_peaks_ws_bytes",
            "hough_vertex_vote", "hough_vertex_peaks", "hough_vertex_table", "hough_vertex_batch_vote_ws_bytes",
            "hough_vertex_batch_peaks_ws_bytes", "hough_vertex_vote_batch", "hough_vertex_peaks_batch"]


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise HoughError(f"{what}: {lib.hough_strerror(rc).decode()} ({rc})")


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise HoughError("device tensor expected")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class Plan:
    """A plan for one detector geometry and parameter grid (owns the sample table)."""

    def __init__(self, cfg, max_hits: Optional[int] = None):
        self.cfg = cfg
        self._r = np.ascontiguousarray(cfg.radii_cm, dtype=np.float64)
        self._hl = np.ascontiguousarray(cfg.halflen_cm, dtype=np.float64)
        geo = Geometry(len(self._r), self._r.ctypes.data_as(C.POINTER(C.c_double)),
                       self._hl.ctypes.data_as(C.POINTER(C.c_double)), cfg.B_tesla)
        self.max_hits = int(max_hits if max_hits is not None else cfg.max_hits_per_event)
        grid = Grid(cfg.n_phi, cfg.n_qpt, cfg.n_d0, cfg.frac_bits, cfg.qpt_min, cfg.qpt_max, cfg.d0_min,
                    cfg.d0_max, cfg.acc_bits, cfg.n_cot, cfg.n_z0, cfg.cot_min, cfg.cot_max, cfg.z0_min,
                    cfg.z0_max, self.max_hits)
        h = C.c_void_p()
        _check(lib.hough_plan_create(C.byref(geo), C.byref(grid), C.byref(h)), "hough_plan_create")
        self.handle = h.value

    def close(self):
        if getattr(self, "handle", None):
            lib.hough_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def acc_bytes(self) -> int:
        return int(lib.hough_acc_bytes(self.handle))

    @property
    def acc_dtype(self):
        return torch.int32 if self.cfg.acc_bits == 32 else torch.int16

    @property
    def angle_bits(self) -> int:
        return int(lib.hough_angle_bits(self.handle))

    def ws_bytes(self, max_peaks: int = 0) -> int:
        return int(lib.hough_event_ws_bytes(self.handle, int(max_peaks)))

    def batch_ws_bytes(self, n_events: int, cap_peaks: int) -> int:
        return int(lib.hough_batch_ws_bytes(self.handle, int(n_events), int(cap_peaks)))

    @property
    def tuning(self) -> dict:
        t = Tuning()
        _check(lib.hough_plan_get_tuning(self.handle, C.byref(t)), "hough_plan_get_tuning")
        return dict(vote_threads=t.vote_threads, vote_grid=t.vote_grid, peak_planes=t.peak_planes,
                    vote_cols=t.vote_cols, assign_blocks=t.assign_blocks, prep_rows=t.prep_rows)

    def set_tuning(self, vote_threads: int = 1024, vote_grid: int = 0, peak_planes: int = 8, vote_cols: int = 0,
                   assign_blocks: int = 0, prep_rows: int = 0) -> None:
        t = Tuning(int(vote_threads), int(vote_grid), int(peak_planes), int(vote_cols), int(assign_blocks),
                   int(prep_rows))
        _check(lib.hough_plan_set_tuning(self.handle, C.byref(t)), "hough_plan_set_tuning")

    def set_vote_events(self, start=None, stop=None) -> None:
        """Have the vote kernel record these torch.cuda.Events (timing enabled) at its own start and
        end; None, None switches it off."""
        def raw(ev):
            if ev is None:
                return None
            if not ev.cuda_event:  # torch creates the HIP event at its first record
                ev.record()
            return ev.cuda_event
        _check(lib.hough_plan_set_vote_events(self.handle, raw(start), raw(stop)), "hough_plan_set_vote_events")

    def set_assign_events(self, start=None, stop=None) -> None:
        """The same for the assignment kernel (plans with the window tables)."""
        def raw(ev):
            if ev is None:
                return None
            if not ev.cuda_event:
                ev.record()
            return ev.cuda_event
        _check(lib.hough_plan_set_assign_events(self.handle, raw(start), raw(stop)), "hough_plan_set_assign_events")

    def table(self) -> np.ndarray:
        c = self.cfg
        out = np.zeros((c.n_layers, c.n_d0, c.n_qpt), dtype=np.int32)
        _check(lib.hough_plan_table(self.handle, out.ctypes.data), "hough_plan_table")
        return out

    @property
    def has_zvote(self) -> bool:
        return self.cfg.n_cot > 0

    def arclen_table(self) -> np.ndarray:
        c = self.cfg
        out = np.zeros((c.n_layers, c.n_d0, c.n_qpt), dtype=np.int32)
        _check(lib.hough_plan_arclen_table(self.handle, out.ctypes.data), "hough_plan_arclen_table")
        return out


def make_hits(x: torch.Tensor, y: torch.Tensor, layer: torch.Tensor, z: Optional[torch.Tensor] = None) -> Hits:
    n = int(x.shape[0])
    for t, dt in ((x, torch.float32), (y, torch.float32), (layer, torch.uint8)):
        if t.dtype != dt or not t.is_contiguous() or int(t.shape[0]) != n:
            raise HoughError("hits must be contiguous float32 x, y and uint8 layer of equal length")
    return Hits(_ptr(x), _ptr(y), _ptr(z), _ptr(layer), n)


def prep(plan: Plan, hits: Hits, phi_out: Optional[torch.Tensor], ws: torch.Tensor, status: torch.Tensor,
         stream=None) -> None:
    _check(lib.hough_prep(plan.handle, C.byref(hits), _ptr(phi_out), _ptr(ws), ws.numel(), _ptr(status),
                          _stream(stream)), "hough_prep")


def vote(plan: Plan, hits: Hits, acc: torch.Tensor, ws: torch.Tensor, status: torch.Tensor, stream=None) -> None:
    if acc.numel() * acc.element_size() < plan.acc_bytes:
        raise HoughError("accumulator too small")
    _check(lib.hough_vote(plan.handle, C.byref(hits), _ptr(acc), _ptr(ws), ws.numel(), _ptr(status),
                          _stream(stream)), "hough_vote")


def vote_cr(plan: Plan, hits: Hits, acc: torch.Tensor, status: torch.Tensor, stream=None) -> None:
    """The vote with each hit's own radius (integer arcsine, every sample computed)."""
    if acc.dtype != torch.int32:
        raise HoughError("hough_vote_cr needs an int32 accumulator")
    _check(lib.hough_vote_cr(plan.handle, C.byref(hits), _ptr(acc), _ptr(status), _stream(stream)), "hough_vote_cr")


def refine(plan: Plan, peaks: torch.Tensor, offsets: torch.Tensor, hit_idx: torch.Tensor, ws: torch.Tensor,
           status: torch.Tensor, window: int, out_hits: torch.Tensor, out_layers: torch.Tensor, stream=None) -> None:
    """Background suppression inside each candidate's bin: per candidate, one hit per layer of the
    densest window of the angle inside the bin (out_hits [cap_peaks][n_layers], out_layers [cap_peaks])."""
    cap_peaks = int(peaks.shape[0])
    if out_hits.numel() < cap_peaks * plan.cfg.n_layers or out_layers.numel() < cap_peaks:
        raise HoughError("out_hits needs [cap_peaks][n_layers] and out_layers [cap_peaks] entries")
    _check(lib.hough_refine(plan.handle, _ptr(peaks), cap_peaks, _ptr(offsets), _ptr(hit_idx), int(hit_idx.numel()),
                            _ptr(ws), ws.numel(), _ptr(status), int(window), _ptr(out_hits), _ptr(out_layers),
                            _stream(stream)), "hough_refine")


def assign_cr_ws_bytes(plan: Plan, cap_peaks: int, cap_pairs: int) -> int:
    return int(lib.hough_assign_cr_ws_bytes(plan.handle, int(cap_peaks), int(cap_pairs)))


def assign_cr(plan: Plan, hits: Hits, peaks: torch.Tensor, offsets: torch.Tensor, hit_idx: torch.Tensor,
              ws: torch.Tensor, ws_cr: torch.Tensor, status: torch.Tensor, stream=None) -> None:
    """Hit lists of the candidates of a per-hit-radius accumulator (after vote_cr and peaks on `ws`)."""
    cap_peaks, cap_pairs = int(peaks.shape[0]), int(hit_idx.numel())
    if offsets.numel() < cap_peaks + 1:
        raise HoughError("offsets must hold cap_peaks + 1 entries")
    _check(lib.hough_assign_cr(plan.handle, C.byref(hits), _ptr(peaks), cap_peaks, _ptr(offsets), _ptr(hit_idx),
                               cap_pairs, _ptr(ws), ws.numel(), _ptr(ws_cr), ws_cr.numel(), _ptr(status),
                               _stream(stream)), "hough_assign_cr")


def vote_prepared(plan: Plan, acc: torch.Tensor, ws: torch.Tensor, status: torch.Tensor, stream=None) -> None:
    if acc.numel() * acc.element_size() < plan.acc_bytes:
        raise HoughError("accumulator too small")
    _check(lib.hough_vote_prepared(plan.handle, _ptr(acc), _ptr(ws), ws.numel(), _ptr(status), _stream(stream)),
           "hough_vote_prepared")


def peaks(plan: Plan, acc: torch.Tensor, threshold: int, out: torch.Tensor, ws: torch.Tensor,
          status: torch.Tensor, stream=None) -> None:
    cap = out.shape[0]
    _check(lib.hough_peaks(plan.handle, _ptr(acc), int(threshold), _ptr(out), int(cap), _ptr(ws), ws.numel(),
                           _ptr(status), _stream(stream)), "hough_peaks")


def assign(plan: Plan, pk: torch.Tensor, offsets: torch.Tensor, hit_idx: torch.Tensor, ws: torch.Tensor,
           status: torch.Tensor, stream=None) -> None:
    cap_peaks = pk.shape[0]
    if offsets.numel() < cap_peaks + 1:
        raise HoughError("offsets needs cap_peaks + 1 entries")
    _check(lib.hough_assign(plan.handle, _ptr(pk), int(cap_peaks), _ptr(offsets), _ptr(hit_idx),
                            int(hit_idx.numel()), _ptr(ws), ws.numel(), _ptr(status), _stream(stream)),
           "hough_assign")


def zvote(plan: Plan, hits: Hits, pk: torch.Tensor, offsets: torch.Tensor, hit_idx: torch.Tensor,
          status: torch.Tensor, out: torch.Tensor, stream=None) -> None:
    cap_peaks = pk.shape[0]
    if offsets.numel() < cap_peaks + 1 or out.numel() < 3 * cap_peaks:
        raise HoughError("offsets needs cap_peaks + 1 entries and out 3 * cap_peaks")
    _check(lib.hough_zvote(plan.handle, C.byref(hits), _ptr(pk), int(cap_peaks), _ptr(offsets), _ptr(hit_idx),
                           int(hit_idx.numel()), _ptr(status), _ptr(out), _stream(stream)), "hough_zvote")


def fit(plan: Plan, hits: Hits, offsets: torch.Tensor, hit_idx: torch.Tensor, status: torch.Tensor,
        out: torch.Tensor, stream=None) -> None:
    """Circle fit of every listed candidate's hit list: out [cap_peaks][4] float64 rows (xc, yc, R^2, n)."""
    cap_peaks = out.shape[0]
    if out.dtype != torch.float64 or out.dim() != 2 or out.shape[1] != 4 or offsets.numel() < cap_peaks + 1:
        raise HoughError("out needs [cap_peaks][4] float64 and offsets cap_peaks + 1 entries")
    _check(lib.hough_fit(plan.handle, C.byref(hits), _ptr(offsets), _ptr(hit_idx), int(cap_peaks),
                         int(hit_idx.numel()), _ptr(status), _ptr(out), _stream(stream)), "hough_fit")


class VertexPlan:
    """The second transform (vertex space) of a first-stage plan; keeps the plan alive."""

    def __init__(self, plan: Plan, n_vr: int, n_vphi: int, r_min: float, r_max: float, min_votes: int):
        self.plan = plan
        self.n_vr, self.n_vphi = int(n_vr), int(n_vphi)
        vg = VertexGrid(self.n_vr, self.n_vphi, float(r_min), float(r_max), int(min_votes))
        h = C.c_void_p()
        _check(lib.hough_vertex_plan_create(plan.handle, C.byref(vg), C.byref(h)), "hough_vertex_plan_create")
        self.handle = h.value

    @classmethod
    def of(cls, plan: Plan) -> "VertexPlan":
        c = plan.cfg
        mv = c.v_min_votes if c.v_min_votes > 0 else c.threshold
        return cls(plan, c.n_vr, c.n_vphi, c.vr_min, c.vr_max, mv)

    def close(self):
        if getattr(self, "handle", None):
            lib.hough_vertex_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def groups(self) -> int:
        return int(lib.hough_vertex_get_groups(self.handle))

    def set_groups(self, groups: int) -> None:
        _check(lib.hough_vertex_set_groups(self.handle, int(groups)), "hough_vertex_set_groups")

    def vote_ws_bytes(self, cap_peaks: int) -> int:
        return int(lib.hough_vertex_vote_ws_bytes(self.handle, int(cap_peaks)))

    def peaks_ws_bytes(self, cap_vpeaks: int) -> int:
        return int(lib.hough_vertex_peaks_ws_bytes(self.handle, int(cap_vpeaks)))

    def table(self) -> np.ndarray:
        c = self.plan.cfg
        out = np.zeros((c.n_d0, c.n_qpt, self.n_vr), dtype=np.int32)
        _check(lib.hough_vertex_table(self.handle, out.ctypes.data), "hough_vertex_table")
        return out


def vertex_vote(vp: VertexPlan, pk: torch.Tensor, status: torch.Tensor, acc_v: torch.Tensor, ws: torch.Tensor,
                status_v: torch.Tensor, stream=None) -> None:
    """Vote the candidates pk [cap][4] (count from the device status) into acc_v [n_vr][n_vphi] int32."""
    if acc_v.dtype != torch.int32 or acc_v.numel() != vp.n_vr * vp.n_vphi or pk.dim() != 2 or pk.shape[1] != 4:
        raise HoughError("acc_v needs n_vr * n_vphi int32 and pk [cap][4]")
    _check(lib.hough_vertex_vote(vp.handle, _ptr(pk), int(pk.shape[0]), _ptr(status), _ptr(acc_v), _ptr(ws),
                                 int(ws.numel() * ws.element_size()), _ptr(status_v), _stream(stream)),
           "hough_vertex_vote")


def vertex_peaks(vp: VertexPlan, acc_v: torch.Tensor, threshold: int, out: torch.Tensor, ws: torch.Tensor,
                 status_v: torch.Tensor, stream=None) -> None:
    if acc_v.dtype != torch.int32 or acc_v.numel() != vp.n_vr * vp.n_vphi:
        raise HoughError("acc_v needs n_vr * n_vphi int32")
    _check(lib.hough_vertex_peaks(vp.handle, _ptr(acc_v), int(threshold), _ptr(out), int(out.shape[0]), _ptr(ws),
                                  int(ws.numel() * ws.element_size()), _ptr(status_v), _stream(stream)),
           "hough_vertex_peaks")


class VertexBuffers:
    """Device buffers of the second transform for one event: vertex accumulator, the two
    workspaces, status and vertex-candidate list."""

    def __init__(self, vp: VertexPlan, cap_peaks: int, cap_vpeaks: int, device="cuda"):
        self.vp = vp
        self.acc = torch.empty((vp.n_vr, vp.n_vphi), dtype=torch.int32, device=device)
        self.ws_vote = torch.empty(max(vp.vote_ws_bytes(cap_peaks), 1), dtype=torch.uint8, device=device)
        self.ws_peaks = torch.empty(vp.peaks_ws_bytes(cap_vpeaks), dtype=torch.uint8, device=device)
        self.status = torch.zeros(STATUS_BYTES // 4, dtype=torch.int32, device=device)
        self.peaks = torch.empty((cap_vpeaks, PEAK_INTS), dtype=torch.int32, device=device)

    def run(self, pk: torch.Tensor, status: torch.Tensor, threshold: int, stream=None) -> None:
        vertex_vote(self.vp, pk, status, self.acc, self.ws_vote, self.status, stream)
        vertex_peaks(self.vp, self.acc, threshold, self.peaks, self.ws_peaks, self.status, stream)

    def results(self) -> dict:
        st = status_dict(self.status)
        n = min(st["n_peaks"], self.peaks.shape[0])
        return dict(status=st, acc=self.acc.cpu().numpy(), peaks=self.peaks[:n].cpu().numpy())


class VertexBatchBuffers:
    """Device buffers of the second transform for a batch: per-event vertex spaces, statuses and
    vertex-candidate lists, and the two workspaces."""

    def __init__(self, vp: VertexPlan, n_events: int, cap_peaks: int, cap_vpeaks: int, device="cuda"):
        self.vp, self.n_events, self.cap_peaks = vp, int(n_events), int(cap_peaks)
        self.acc = torch.empty((n_events, vp.n_vr, vp.n_vphi), dtype=torch.int32, device=device)
        self.ws_vote = torch.empty(int(lib.hough_vertex_batch_vote_ws_bytes(vp.handle, n_events, cap_peaks)),
                                   dtype=torch.uint8, device=device)
        self.ws_peaks = torch.empty(int(lib.hough_vertex_batch_peaks_ws_bytes(vp.handle, n_events, cap_vpeaks)),
                                    dtype=torch.uint8, device=device)
        self.status = torch.zeros((n_events, STATUS_BYTES // 4), dtype=torch.int32, device=device)
        self.peaks = torch.empty((n_events, cap_vpeaks, PEAK_INTS), dtype=torch.int32, device=device)

    def run(self, pk: torch.Tensor, status: torch.Tensor, threshold: int, stream=None) -> None:
        """pk: [n_events * cap_peaks][4] (or [n_events][cap_peaks][4]) candidate lists; status: the
        per-event statuses of the first stage."""
        if pk.numel() != self.n_events * self.cap_peaks * 4:
            raise HoughError("pk needs n_events * cap_peaks rows")
        _check(lib.hough_vertex_vote_batch(self.vp.handle, self.n_events, _ptr(pk), self.cap_peaks, _ptr(status),
                                           _ptr(self.acc), _ptr(self.ws_vote), int(self.ws_vote.numel()),
                                           _ptr(self.status), _stream(stream)), "hough_vertex_vote_batch")
        _check(lib.hough_vertex_peaks_batch(self.vp.handle, self.n_events, _ptr(self.acc), int(threshold),
                                            _ptr(self.peaks), int(self.peaks.shape[1]), _ptr(self.ws_peaks),
                                            int(self.ws_peaks.numel()), _ptr(self.status), _stream(stream)),
               "hough_vertex_peaks_batch")

    def results(self, e: int) -> dict:
        st = status_dict(self.status[e])
        n = min(st["n_peaks"], self.peaks.shape[1])
        return dict(status=st, acc=self.acc[e].cpu().numpy(), peaks=self.peaks[e, :n].cpu().numpy())


def status_dict(status: torch.Tensor) -> dict:
    b = status.detach().to("cpu").numpy().view(np.uint8)[:STATUS_BYTES].tobytes()
    n_hits, n_bad = np.frombuffer(b[0:8], dtype=np.int32)
    (n_votes,) = np.frombuffer(b[8:16], dtype=np.int64)
    n_peaks, flags = np.frombuffer(b[16:24], dtype=np.int32)
    (n_pairs,) = np.frombuffer(b[24:32], dtype=np.int64)
    return dict(n_hits=int(n_hits), n_bad_hits=int(n_bad), n_votes=int(n_votes), n_peaks=int(n_peaks),
                flags=int(flags), n_pairs=int(n_pairs))


class EventBuffers:
    """Device buffers for one event of a plan: accumulator, workspace, status,
    candidate list and CSR hit lists (caller-owned memory, reused per event)."""

    def __init__(self, plan: Plan, cap_peaks: int, cap_pairs: int, device="cuda"):
        self.plan = plan
        c = plan.cfg
        self.acc = torch.empty((c.n_d0, c.n_qpt, c.n_phi), dtype=plan.acc_dtype, device=device)
        self.ws = torch.empty(plan.ws_bytes(cap_peaks), dtype=torch.uint8, device=device)
        self.status = torch.zeros(STATUS_BYTES // 4, dtype=torch.int32, device=device)
        self.peaks = torch.empty((cap_peaks, PEAK_INTS), dtype=torch.int32, device=device)
        self.offsets = torch.empty(cap_peaks + 1, dtype=torch.int32, device=device)
        self.hit_idx = torch.empty(cap_pairs, dtype=torch.int32, device=device)
        self.zv = torch.empty((cap_peaks, 3), dtype=torch.int32, device=device) if plan.has_zvote else None
        self.fit = None  # [cap_peaks][4] float64 once run_fit has been called

    def run_fit(self, hits: Hits, stream=None) -> None:
        """The circle fit of every listed candidate (after run)."""
        if self.fit is None:
            self.fit = torch.empty((self.peaks.shape[0], 4), dtype=torch.float64, device=self.peaks.device)
        fit(self.plan, hits, self.offsets, self.hit_idx, self.status, self.fit, stream)

    def run(self, hits: Hits, threshold: int, stream=None, do_assign: bool = True) -> None:
        vote(self.plan, hits, self.acc, self.ws, self.status, stream)
        peaks(self.plan, self.acc, threshold, self.peaks, self.ws, self.status, stream)
        if do_assign:
            assign(self.plan, self.peaks, self.offsets, self.hit_idx, self.ws, self.status, stream)
            if self.zv is not None and hits.z:
                zvote(self.plan, hits, self.peaks, self.offsets, self.hit_idx, self.status, self.zv, stream)

    def results(self) -> dict:
        st = status_dict(self.status)
        n = min(st["n_peaks"], self.peaks.shape[0])
        pk = self.peaks[:n].cpu().numpy()
        offs = self.offsets[: n + 1].cpu().numpy().astype(np.int64)
        npairs = min(st["n_pairs"], self.hit_idx.numel())
        hit_idx = self.hit_idx[:npairs].cpu().numpy()
        out = dict(status=st, peaks=pk, offsets=offs, hit_idx=hit_idx)
        if self.zv is not None:
            out["zvote"] = self.zv[:n].cpu().numpy()
        if self.fit is not None:
            out["fit"] = self.fit[:n].cpu().numpy()
        return out


def hits_to_device(ev, device="cuda"):
    x = torch.from_numpy(np.ascontiguousarray(ev.x)).to(device)
    y = torch.from_numpy(np.ascontiguousarray(ev.y)).to(device)
    lay = torch.from_numpy(np.ascontiguousarray(ev.layer)).to(device)
    z = torch.from_numpy(np.ascontiguousarray(ev.z)).to(device) if getattr(ev, "z", None) is not None else None
    return x, y, lay, z


def run_batch(plan: Plan, b: Batch, stream=None) -> None:
    """hough_run_batch on a Batch whose pointers the caller set (e.g. outputs in slots of a larger arena)."""
    _check(lib.hough_run_batch(plan.handle, C.byref(b), _stream(stream)), "hough_run_batch")


class BatchBuffers:
    """Device buffers of a batch of up to `n_events` events (packed hits and strided outputs)."""

    def __init__(self, plan: Plan, n_events: int, max_total_hits: int, cap_peaks: int, cap_pairs: int,
                 device="cuda"):
        self.plan = plan
        c = plan.cfg
        self.n_events = int(n_events)
        self.cap_peaks, self.cap_pairs = int(cap_peaks), int(cap_pairs)
        self.x = torch.zeros(max(max_total_hits, 1), dtype=torch.float32, device=device)
        self.y = torch.zeros_like(self.x)
        self.z = torch.zeros_like(self.x) if plan.has_zvote else None
        self.layer = torch.zeros(max(max_total_hits, 1), dtype=torch.uint8, device=device)
        self.hit_offsets = torch.zeros(self.n_events + 1, dtype=torch.int32, device=device)
        self.acc = torch.empty((self.n_events, c.n_d0, c.n_qpt, c.n_phi), dtype=plan.acc_dtype, device=device)
        self.peaks = torch.empty((self.n_events, cap_peaks, PEAK_INTS), dtype=torch.int32, device=device)
        self.offsets = torch.empty((self.n_events, cap_peaks + 1), dtype=torch.int32, device=device)
        self.hit_idx = torch.empty((self.n_events, cap_pairs), dtype=torch.int32, device=device)
        self.ws = torch.empty(plan.batch_ws_bytes(self.n_events, cap_peaks), dtype=torch.uint8, device=device)
        self.status = torch.zeros((self.n_events, STATUS_BYTES // 4), dtype=torch.int32, device=device)
        self.zv = (torch.empty((self.n_events, cap_peaks, 3), dtype=torch.int32, device=device)
                   if plan.has_zvote else None)
        self.fit = None  # [n_events][cap_peaks][4] float64 once run_fit has been called

    def load(self, events, stream=None) -> None:
        """Copy the packed hits of `events` (at most n_events) into the device buffers."""
        assert len(events) == self.n_events
        offs = np.zeros(len(events) + 1, dtype=np.int32)
        offs[1:] = np.cumsum([e.n for e in events])
        n = int(offs[-1])
        assert n <= self.x.numel()
        if n:
            self.x[:n].copy_(torch.from_numpy(np.concatenate([e.x for e in events])), non_blocking=False)
            self.y[:n].copy_(torch.from_numpy(np.concatenate([e.y for e in events])), non_blocking=False)
            self.layer[:n].copy_(torch.from_numpy(np.concatenate([e.layer for e in events])), non_blocking=False)
            if self.z is not None:
                self.z[:n].copy_(torch.from_numpy(np.concatenate([e.z for e in events]).astype(np.float32)))
        self.hit_offsets.copy_(torch.from_numpy(offs))

    def struct(self, threshold: int, n_events: Optional[int] = None, zvote: bool = True) -> Batch:
        n_events = self.n_events if n_events is None else int(n_events)
        if not 1 <= n_events <= self.n_events:
            raise HoughError("n_events out of range")
        return Batch(_ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(self.layer), _ptr(self.hit_offsets), n_events,
                     int(threshold), self.cap_peaks, self.cap_pairs, _ptr(self.acc), _ptr(self.peaks),
                     _ptr(self.offsets), _ptr(self.hit_idx), _ptr(self.ws), self.ws.numel(), _ptr(self.status),
                     _ptr(self.zv) if zvote else None)

    def run(self, threshold: int, stream=None, n_events: Optional[int] = None, zvote: bool = True) -> None:
        b = self.struct(threshold, n_events, zvote)
        _check(lib.hough_run_batch(self.plan.handle, C.byref(b), _stream(stream)), "hough_run_batch")

    def run_noalloc(self, threshold: int, stream=None, n_events: Optional[int] = None, zvote: bool = True) -> None:
        """The same chain through hough_run_batch_noalloc: the library's scratch array is the workspace
        (this object's `ws` is not used)."""
        b = self.struct(threshold, n_events, zvote)
        b.ws, b.ws_bytes = None, 0
        _check(lib.hough_run_batch_noalloc(self.plan.handle, C.byref(b), _stream(stream)),
               "hough_run_batch_noalloc")

    def run_fit(self, stream=None, n_events: Optional[int] = None) -> None:
        """Circle fit of every listed candidate of every event (after run)."""
        if self.fit is None:
            self.fit = torch.empty((self.n_events, self.cap_peaks, 4), dtype=torch.float64, device=self.x.device)
        b = self.struct(1, n_events)
        _check(lib.hough_fit_batch(self.plan.handle, C.byref(b), _ptr(self.fit), _stream(stream)), "hough_fit_batch")

    def results(self, e: int) -> dict:
        st = status_dict(self.status[e])
        n = min(st["n_peaks"], self.cap_peaks)
        pk = self.peaks[e, :n].cpu().numpy()
        offs = self.offsets[e, : n + 1].cpu().numpy().astype(np.int64)
        npairs = min(st["n_pairs"], self.cap_pairs)
        out = dict(status=st, peaks=pk, offsets=offs, hit_idx=self.hit_idx[e, :npairs].cpu().numpy())
        if self.zv is not None:
            out["zvote"] = self.zv[e, :n].cpu().numpy()
        if self.fit is not None:
            out["fit"] = self.fit[e, :n].cpu().numpy()
        return out


class Graph:
    """The batched chain of a BatchBuffers captured into a hipGraph (buffers bound at capture)."""

    def __init__(self, bufs: BatchBuffers, threshold: int, stream):
        self.bufs = bufs
        self._b = bufs.struct(threshold)
        h = C.c_void_p()
        _check(lib.hough_batch_graph_create(bufs.plan.handle, C.byref(self._b), _stream(stream), C.byref(h)),
               "hough_batch_graph_create")
        self.handle = h.value

    def launch(self, stream=None) -> None:
        _check(lib.hough_graph_launch(self.handle, _stream(stream)), "hough_graph_launch")

    def close(self):
        if getattr(self, "handle", None):
            lib.hough_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
