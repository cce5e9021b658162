"""ctypes binding of the roofline micro-benchmarks (libroofline_probe.so): the measured rates the
kernels' roofline fractions are taken against.

    lds(kind)  conflict-free LDS operations of 64-lane waves, 16 independent instructions per loop
               iteration: "atomic" (ds_add_u32, no return), "read32", "write32", "read128",
               "atomic_rtn" (ds_add_rtn_u32), "vote_pair" (add with return + subtract of one word)
    hbm(kind)  streaming "copy" (bytes read + written) or "fill" (bytes written) of a large buffer
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libroofline_probe.so")
LDS_KINDS = {"atomic": 0, "read32": 1, "write32": 2, "read128": 3, "atomic_rtn": 4, "vote_pair": 5}
HBM_KINDS = {"copy": 0, "fill": 1}
LDS_BYTES = {"atomic": 4, "read32": 4, "write32": 4, "read128": 16, "atomic_rtn": 4, "vote_pair": 4}


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    L.probe_lds.restype = C.c_int
    L.probe_lds.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_double),
                            C.POINTER(C.c_float)]
    L.probe_hbm.restype = C.c_int
    L.probe_hbm.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.POINTER(C.c_double),
                            C.POINTER(C.c_float)]
    return L


lib = _load()


def lds(kind: str, blocks: int, iters: int = 4096, reps: int = 5) -> dict:
    """Rate of one LDS operation kind over `blocks` workgroups of 1024 threads."""
    out = torch.zeros(blocks * 1024, dtype=torch.int32, device="cuda")
    ops, us = C.c_double(), C.c_float()
    if lib.probe_lds(LDS_KINDS[kind], int(blocks), int(iters), int(reps), C.c_void_p(out.data_ptr()), C.byref(ops),
                     C.byref(us)) != 0:
        raise RuntimeError(f"probe_lds({kind}) failed")
    if int(out.count_nonzero()) != 0:
        raise RuntimeError(f"probe_lds({kind}): the kernel's own check failed")
    rate = ops.value / (us.value * 1e-6)
    return {"kind": kind, "blocks": blocks, "lane_ops_per_launch": ops.value, "us_per_launch": round(us.value, 3),
            "lane_ops_per_s": rate, "bytes_per_s": rate * LDS_BYTES[kind]}


def hbm(kind: str, nbytes: int = 2 << 30, blocks: int = 4096, reps: int = 10) -> dict:
    """Streaming bandwidth of a plain copy or fill of `nbytes` bytes."""
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda") if kind == "copy" else None
    if src is not None:
        src.fill_(1)
    moved, us = C.c_double(), C.c_float()
    if lib.probe_hbm(HBM_KINDS[kind], C.c_void_p(src.data_ptr()) if src is not None else None,
                     C.c_void_p(dst.data_ptr()), nbytes, int(blocks), int(reps), C.byref(moved), C.byref(us)) != 0:
        raise RuntimeError(f"probe_hbm({kind}) failed")
    return {"kind": kind, "bytes": nbytes, "blocks": blocks, "us_per_launch": round(us.value, 2),
            "bytes_moved_per_launch": moved.value, "gb_per_s": round(moved.value / (us.value * 1e-6) / 1e9, 1)}
