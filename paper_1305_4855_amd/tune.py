"""Launch-shape autotuner for the batched chain.

Times the whole batched chain (prep -> persistent vote -> peaks -> assign) on a
representative batch for every candidate launch shape (vote workgroup size,
number of persistent vote workgroups, d0 planes per peak-finder thread), and
stores the fastest in tuning_cache.json, keyed by device architecture and grid.
Every shape gives bit-identical results; only the time differs.

    python -m paper_1305_4855_amd.tune --config c3 --events 64
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")

CANDIDATES = dict(vote_threads=(512, 1024), vote_grid=(256, 512, 1024), peak_planes=(8, 16, 32))


def cache_key(cfg, arch: str) -> str:
    return f"{arch}:{cfg.n_phi}x{cfg.n_qpt}x{cfg.n_d0}:i{cfg.acc_bits}"


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def apply(plan) -> dict:
    """Set the cached tuning for this plan's grid on this device, if there is one."""
    entry = load_cache().get(cache_key(plan.cfg, device_arch()))
    if entry:
        plan.set_tuning(**entry["best"])
    return plan.tuning


def tune(cfg, events, reps: int = 3, log=print) -> dict:
    import torch

    from . import hough as H

    plan = H.Plan(cfg, max_hits=cfg.max_hits_per_event)
    total = sum(e.n for e in events)
    bufs = H.BatchBuffers(plan, len(events), total, cap_peaks=1 << 19, cap_pairs=1 << 24)
    bufs.load(events)
    stream = torch.cuda.current_stream()
    results = []
    ref = None
    for vt, vg, pp in itertools.product(*CANDIDATES.values()):
        t = dict(vote_threads=vt, vote_grid=vg, peak_planes=pp)
        plan.set_tuning(**t)
        bufs.run(cfg.threshold, stream)
        torch.cuda.synchronize()
        st = bufs.status.cpu().numpy().copy()
        if ref is None:
            ref = st
        elif not (st == ref).all():
            raise RuntimeError(f"results differ for launch shape {t}")
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            bufs.run(cfg.threshold, stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        results.append((ms, t))
        log(f"  {t}: {ms:.3f} ms per batch of {len(events)}")
    results.sort(key=lambda r: r[0])
    return dict(best=results[0][1], best_ms=round(results[0][0], 4), n_events=len(events),
                table=[dict(ms=round(ms, 4), **t) for ms, t in results], when=time.strftime("%Y-%m-%d %H:%M:%S"))


def main() -> int:
    from . import configs, synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c3")
    ap.add_argument("--events", type=int, default=64)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    cfg = configs.get(args.config)
    events = [synth.make_event(cfg, i) for i in range(args.events)]
    arch = device_arch()
    print(f"tuning {cfg.name} on {arch} with {len(events)} events", flush=True)
    entry = tune(cfg, events, reps=args.reps, log=lambda s: print(s, flush=True))
    cache = load_cache()
    cache[cache_key(cfg, arch)] = entry
    with open(CACHE, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    print(json.dumps({"key": cache_key(cfg, arch), "best": entry["best"], "best_ms": entry["best_ms"]}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
