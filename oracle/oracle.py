"""ctypes wrapper of the CPU oracle (hough_oracle.c).

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It imports nothing from
the GPU package; configurations are taken by duck typing (any object with the
geometry and grid attributes).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hough_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# IEEE double semantics: no contraction into fused multiply-add, no fast-math.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Cfg(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32), ("r_cm", C.POINTER(C.c_double)), ("halflen_cm", C.POINTER(C.c_double)),
        ("B_tesla", C.c_double),
        ("n_phi", C.c_int32), ("n_qpt", C.c_int32), ("n_d0", C.c_int32), ("frac_bits", C.c_int32),
        ("qpt_min", C.c_double), ("qpt_max", C.c_double), ("d0_min", C.c_double), ("d0_max", C.c_double),
        ("n_cot", C.c_int32), ("n_z0", C.c_int32),
        ("cot_min", C.c_double), ("cot_max", C.c_double), ("z0_min", C.c_double), ("z0_max", C.c_double),
    ]


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = load(LIB)
    return _lib


def use_library(path: Optional[str]) -> None:
    """Point the wrapper at another build of the oracle source (the mutation
    tests compile deliberately broken copies to show the pins catch them)."""
    global _lib
    _lib = load(path) if path else None


def load(path: str) -> C.CDLL:
    L = C.CDLL(path)
    P = C.c_void_p
    L.or_q16.restype = C.c_int32; L.or_q16.argtypes = [C.c_float]
    L.or_azimuth.restype = C.c_uint32; L.or_azimuth.argtypes = [C.c_int32, C.c_int32]
    L.or_hit.restype = C.c_int
    L.or_hit.argtypes = [C.c_float, C.c_float, C.c_uint8, C.c_int32, P, P]
    L.or_prep.restype = None; L.or_prep.argtypes = [C.c_int32, P, P, P, C.c_int32, P, P]
    L.or_angle_bits.restype = C.c_int32; L.or_angle_bits.argtypes = [P]
    L.or_qpt_centre.restype = C.c_double; L.or_qpt_centre.argtypes = [P, C.c_int32]
    L.or_d0_centre.restype = C.c_double; L.or_d0_centre.argtypes = [P, C.c_int32]
    L.or_curvature.restype = C.c_double; L.or_curvature.argtypes = [P, C.c_int32]
    L.or_sample.restype = C.c_int
    L.or_sample.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, P]
    L.or_vote.restype = C.c_int64; L.or_vote.argtypes = [P, C.c_int32, P, P, P, P]
    L.or_vote_columns.restype = None
    L.or_vote_columns.argtypes = [P, C.c_int32, P, P, P, C.c_int32, P, P]
    L.or_peaks.restype = C.c_int64; L.or_peaks.argtypes = [P, P, C.c_int32, C.c_int64, P]
    L.or_peak_at.restype = C.c_int
    L.or_peak_at.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    L.or_assign.restype = C.c_int64
    L.or_assign.argtypes = [P, C.c_int32, P, P, P, C.c_int32, P, P, P, C.c_int64]
    L.or_arclen.restype = C.c_int
    L.or_arclen.argtypes = [C.c_double, C.c_double, C.c_double, P]
    L.or_cot_centre_q16.restype = C.c_int64; L.or_cot_centre_q16.argtypes = [P, C.c_int32]
    L.or_zvote.restype = None
    L.or_zvote.argtypes = [P, C.c_int32, P, P, C.c_int32, P, P, P, P]
    L.or_fit.restype = None
    L.or_fit.argtypes = [P, P, C.c_int32, P, P, P]
    L.or_isqrt.restype = C.c_uint64; L.or_isqrt.argtypes = [C.c_uint64]
    L.or_sample_cr.restype = C.c_int
    L.or_sample_cr.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, P]
    L.or_hit_radius.restype = C.c_double; L.or_hit_radius.argtypes = [C.c_int32, C.c_int32]
    L.or_vote_cr.restype = C.c_int64; L.or_vote_cr.argtypes = [P, C.c_int32, P, P, P, P]
    L.or_set_threads.restype = C.c_int; L.or_set_threads.argtypes = [C.c_int]
    L.or_refine.restype = C.c_int64
    L.or_refine.argtypes = [P, C.c_int32, P, P, P, C.c_int32, P, P, P, C.c_int32, P, P]
    L.or_assign_cr.restype = C.c_int64
    L.or_assign_cr.argtypes = [P, C.c_int32, P, P, P, C.c_int32, P, P, P, C.c_int64]
    L.or_vertex_radius.restype = C.c_double
    L.or_vertex_radius.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_int32]
    L.or_vertex_vote.restype = C.c_int64
    L.or_vertex_vote.argtypes = [P, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_int32, P, P]
    return L


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


class Cfg:
    """Oracle view of a workload configuration (keeps its arrays alive)."""

    def __init__(self, cfg):
        self.src = cfg
        self._r = np.ascontiguousarray(cfg.radii_cm, dtype=np.float64)
        self._hl = np.ascontiguousarray(cfg.halflen_cm, dtype=np.float64)
        self.s = _Cfg(
            n_layers=len(self._r), r_cm=self._r.ctypes.data_as(C.POINTER(C.c_double)),
            halflen_cm=self._hl.ctypes.data_as(C.POINTER(C.c_double)), B_tesla=cfg.B_tesla,
            n_phi=cfg.n_phi, n_qpt=cfg.n_qpt, n_d0=cfg.n_d0, frac_bits=cfg.frac_bits,
            qpt_min=cfg.qpt_min, qpt_max=cfg.qpt_max, d0_min=cfg.d0_min, d0_max=cfg.d0_max,
            n_cot=cfg.n_cot, n_z0=cfg.n_z0, cot_min=cfg.cot_min, cot_max=cfg.cot_max,
            z0_min=cfg.z0_min, z0_max=cfg.z0_max)
        self.n_phi, self.n_qpt, self.n_d0 = cfg.n_phi, cfg.n_qpt, cfg.n_d0

    @property
    def ptr(self) -> int:
        return C.addressof(self.s)


def _hits(ev):
    x = np.ascontiguousarray(ev.x, dtype=np.float32)
    y = np.ascontiguousarray(ev.y, dtype=np.float32)
    lay = np.ascontiguousarray(ev.layer, dtype=np.uint8)
    return x, y, lay


# ---------------------------------------------------------------- scalar steps
def q16(v: float) -> int:
    return int(lib().or_q16(float(v)))


def azimuth(X: int, Y: int) -> int:
    return int(lib().or_azimuth(int(X), int(Y)))


def hit(x: float, y: float, layer: int, n_layers: int):
    X = C.c_int32(); Y = C.c_int32()
    ok = lib().or_hit(float(x), float(y), int(layer), int(n_layers), C.addressof(X), C.addressof(Y))
    return bool(ok), X.value, Y.value


def sample(r: float, c: float, d: float, M: int):
    E = C.c_int32()
    ok = lib().or_sample(float(r), float(c), float(d), int(M), C.addressof(E))
    return bool(ok), E.value


def arclen(r: float, c: float, d: float):
    S = C.c_int64()
    ok = lib().or_arclen(float(r), float(c), float(d), C.addressof(S))
    return bool(ok), S.value


def angle_bits(cfg: Cfg) -> int:
    return int(lib().or_angle_bits(cfg.ptr))


def qpt_centre(cfg: Cfg, k: int) -> float:
    return float(lib().or_qpt_centre(cfg.ptr, k))


def d0_centre(cfg: Cfg, l: int) -> float:
    return float(lib().or_d0_centre(cfg.ptr, l))


def curvature(cfg: Cfg, k: int) -> float:
    return float(lib().or_curvature(cfg.ptr, k))


def cot_centre_q16(cfg: Cfg, m: int) -> int:
    return int(lib().or_cot_centre_q16(cfg.ptr, m))


# ---------------------------------------------------------------- event steps
def prep(ev, n_layers: int):
    x, y, lay = _hits(ev)
    n = x.shape[0]
    phi = np.zeros(n, dtype=np.uint32)
    ok = np.zeros(n, dtype=np.uint8)
    lib().or_prep(n, _p(x), _p(y), _p(lay), n_layers, _p(phi), _p(ok))
    return phi, ok.astype(bool)


def vote(cfg: Cfg, ev):
    x, y, lay = _hits(ev)
    acc = np.zeros((cfg.n_d0, cfg.n_qpt, cfg.n_phi), dtype=np.int32)
    nv = lib().or_vote(cfg.ptr, x.shape[0], _p(x), _p(y), _p(lay), _p(acc))
    return acc, int(nv)


def vote_columns(cfg: Cfg, ev, cols: np.ndarray):
    x, y, lay = _hits(ev)
    cols = np.ascontiguousarray(cols, dtype=np.int32).reshape(-1, 2)
    out = np.zeros((cols.shape[0], cfg.n_phi), dtype=np.int32)
    lib().or_vote_columns(cfg.ptr, x.shape[0], _p(x), _p(y), _p(lay), cols.shape[0], _p(cols), _p(out))
    return out


def peaks(cfg: Cfg, acc: np.ndarray, thr: int, cap: int = 1 << 24):
    acc = np.ascontiguousarray(acc, dtype=np.int32)
    assert acc.size == cfg.n_d0 * cfg.n_qpt * cfg.n_phi
    out = np.zeros((cap, 4), dtype=np.int32)
    n = int(lib().or_peaks(cfg.ptr, _p(acc), int(thr), int(cap), _p(out)))
    return n, out[: min(n, cap)].copy()


def peak_at(cfg: Cfg, acc: np.ndarray, l: int, k: int, b: int, thr: int) -> bool:
    acc = np.ascontiguousarray(acc, dtype=np.int32)
    return bool(lib().or_peak_at(cfg.ptr, _p(acc), l, k, b, int(thr)))


def assign(cfg: Cfg, ev, pk: np.ndarray, cap_pairs: int = 1 << 26):
    x, y, lay = _hits(ev)
    pk = np.ascontiguousarray(pk, dtype=np.int32).reshape(-1, 4)
    offs = np.zeros(pk.shape[0] + 1, dtype=np.int64)
    total_guess = int(pk[:, 3].sum()) if pk.shape[0] else 0
    cap = min(int(cap_pairs), max(total_guess, 1))
    hit_idx = np.zeros(max(cap, 1), dtype=np.int32)
    tot = int(lib().or_assign(cfg.ptr, x.shape[0], _p(x), _p(y), _p(lay), pk.shape[0], _p(pk),
                              _p(offs), _p(hit_idx), cap))
    return offs, hit_idx[: min(tot, cap)].copy(), tot


def zvote(cfg: Cfg, ev, pk: np.ndarray, offs: np.ndarray, hit_idx: np.ndarray):
    assert ev.z is not None
    z = np.ascontiguousarray(ev.z, dtype=np.float32)
    lay = np.ascontiguousarray(ev.layer, dtype=np.uint8)
    pk = np.ascontiguousarray(pk, dtype=np.int32).reshape(-1, 4)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    hit_idx = np.ascontiguousarray(hit_idx, dtype=np.int32)
    out = np.zeros((pk.shape[0], 3), dtype=np.int32)
    lib().or_zvote(cfg.ptr, z.shape[0], _p(z), _p(lay), pk.shape[0], _p(pk), _p(offs), _p(hit_idx), _p(out))
    return out


def fit(ev, offs: np.ndarray, hit_idx: np.ndarray) -> np.ndarray:
    """Algebraic (Kasa) circle fit of each candidate's hit list: rows (xc, yc, R^2, n_hits);
    R^2 = -1 for fewer than 3 hits or a singular system."""
    x, y, _ = _hits(ev)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    hit_idx = np.ascontiguousarray(hit_idx, dtype=np.int32)
    n = offs.shape[0] - 1
    out = np.zeros((max(n, 0), 4), dtype=np.float64)
    if n > 0:
        lib().or_fit(_p(x), _p(y), n, _p(offs), _p(hit_idx), _p(out))
    return out


def fit_points(x, y) -> np.ndarray:
    """The fit of one list made of the given points (float32 coordinates)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    offs = np.array([0, x.shape[0]], dtype=np.int64)
    idx = np.arange(x.shape[0], dtype=np.int32)
    out = np.zeros((1, 4), dtype=np.float64)
    lib().or_fit(_p(x), _p(y), 1, _p(offs), _p(idx if idx.size else np.zeros(1, np.int32)), _p(out))
    return out[0]



# ---------------------------------------------------------------- second transform (vertices)
class VertexGrid:
    """Vertex space of the second transform: n_vr radius rows over [r_min, r_max) cm times
    n_vphi azimuth bins; candidates with fewer than min_votes first-stage votes do not vote."""

    def __init__(self, n_vr: int, n_vphi: int, r_min: float, r_max: float, min_votes: int = 1):
        self.n_vr, self.n_vphi = int(n_vr), int(n_vphi)
        self.r_min, self.r_max = float(r_min), float(r_max)
        self.min_votes = int(min_votes)

    @classmethod
    def of(cls, cfg) -> "VertexGrid":
        mv = cfg.v_min_votes if cfg.v_min_votes > 0 else cfg.threshold
        return cls(cfg.n_vr, cfg.n_vphi, cfg.vr_min, cfg.vr_max, mv)


def vertex_radius(vg: VertexGrid, j: int) -> float:
    return float(lib().or_vertex_radius(vg.n_vr, vg.r_min, vg.r_max, int(j)))


def vertex_vote(cfg: Cfg, vg: VertexGrid, pk: np.ndarray):
    """Vertex accumulator acc_v[n_vr][n_vphi] of a candidate list (rows l, k, b, votes)."""
    pk = np.ascontiguousarray(pk, dtype=np.int32).reshape(-1, 4)
    acc = np.zeros((vg.n_vr, vg.n_vphi), dtype=np.int32)
    nv = lib().or_vertex_vote(cfg.ptr, vg.n_vr, vg.n_vphi, vg.r_min, vg.r_max, vg.min_votes, pk.shape[0],
                              _p(pk if pk.size else np.zeros(4, np.int32)), _p(acc))
    return acc, int(nv)


def vertex_peaks(vg: VertexGrid, acc_v: np.ndarray, thr: int, cap: int = 1 << 20):
    """Local maxima of the vertex space: the peak rule of the first transform on the grid
    (1 x n_vr x n_vphi).  Rows (0, j, azimuth bin, votes)."""
    acc_v = np.ascontiguousarray(acc_v, dtype=np.int32)
    assert acc_v.size == vg.n_vr * vg.n_vphi
    g = _Cfg(n_layers=0, B_tesla=0.0, n_phi=vg.n_vphi, n_qpt=vg.n_vr, n_d0=1, frac_bits=0,
             qpt_min=0.0, qpt_max=0.0, d0_min=0.0, d0_max=0.0, n_cot=0, n_z0=0,
             cot_min=0.0, cot_max=0.0, z0_min=0.0, z0_max=0.0)
    out = np.zeros((cap, 4), dtype=np.int32)
    n = int(lib().or_peaks(C.addressof(g), _p(acc_v), int(thr), int(cap), _p(out)))
    return n, out[: min(n, cap)].copy()


# ---------------------------------------------------------------- per-hit radius transform
def isqrt(v: int) -> int:
    return int(lib().or_isqrt(int(v)))


def sample_cr(r: float, c: float, d: float, M: int):
    E = C.c_int32()
    ok = lib().or_sample_cr(float(r), float(c), float(d), int(M), C.addressof(E))
    return bool(ok), E.value


def hit_radius(X: int, Y: int) -> float:
    return float(lib().or_hit_radius(int(X), int(Y)))


def vote_cr(cfg: Cfg, ev):
    """Accumulator of the transform with each hit's own radius (integer arcsine)."""
    x, y, lay = _hits(ev)
    acc = np.zeros((cfg.n_d0, cfg.n_qpt, cfg.n_phi), dtype=np.int32)
    nv = lib().or_vote_cr(cfg.ptr, x.shape[0], _p(x), _p(y), _p(lay), _p(acc))
    return acc, int(nv)


def assign_cr(cfg: Cfg, ev, pk: np.ndarray, cap_pairs: int = 1 << 26):
    """Hit lists of candidates of the per-hit-radius transform (same CSR layout and order as assign)."""
    x, y, lay = _hits(ev)
    pk = np.ascontiguousarray(pk, dtype=np.int32).reshape(-1, 4)
    offs = np.zeros(pk.shape[0] + 1, dtype=np.int64)
    total_guess = int(pk[:, 3].sum()) if pk.shape[0] else 0
    cap = min(int(cap_pairs), max(total_guess, 1))
    hit_idx = np.zeros(max(cap, 1), dtype=np.int32)
    tot = int(lib().or_assign_cr(cfg.ptr, x.shape[0], _p(x), _p(y), _p(lay), pk.shape[0], _p(pk),
                                 _p(offs), _p(hit_idx), cap))
    return offs, hit_idx[: min(tot, cap)].copy(), tot


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops (0: leave as is); returns the count in effect."""
    return int(lib().or_set_threads(int(n)))


def refine(cfg: Cfg, ev, pk: np.ndarray, offs: np.ndarray, hit_idx: np.ndarray, w: int):
    """Refined lists of candidates (background suppression inside the bin): ([n][n_layers] hit or -1,
    [n] layers covered)."""
    x, y, lay = _hits(ev)
    pk = np.ascontiguousarray(pk, dtype=np.int32).reshape(-1, 4)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    hit_idx = np.ascontiguousarray(hit_idx, dtype=np.int32)
    n = pk.shape[0]
    nl = len(cfg.src.radii_cm)
    out = np.full((max(n, 1), nl), -1, dtype=np.int32)
    layers = np.zeros(max(n, 1), dtype=np.int32)
    lib().or_refine(cfg.ptr, x.shape[0], _p(x), _p(y), _p(lay), n, _p(pk), _p(offs), _p(hit_idx), int(w),
                    _p(out), _p(layers))
    return out[:n], layers[:n]
