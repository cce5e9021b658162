"""Autotuner of the tile shapes and launch shapes of the hot path.

The knobs (all in hough_tuning_t; every value gives bit-identical results, only the time differs):
  vote_cols      columns of the accumulator per work item of the table vote (a tile of the vote)
  vote_grid      persistent workgroups pulling (event, column tile) items from the batch's queue
  vote_threads   workgroup size of the LDS-slab vote (plans without the window tables)
  peak_planes    d0 planes one peak-finder thread walks (the depth of a marking tile)
  assign_blocks  assignment workgroups per event
  prep_rows      phi0 rows per workgroup of the sorting/table pass (the prep tile)

For a workload, the tuner times the chain on representative events for every value of one knob
at a time, keeps the fastest, and sweeps all knobs twice (coordinate descent).  Before timing a
shape it checks that the shape's outputs (accumulators, candidate lists, CSR offsets and hit
lists, statuses, r-z results) have the same checksums as the first shape's.  The best shape is
stored in tuning_cache.json under a key of device architecture, grid, counter width, angle bits,
kernel path and mode ("batch": the batched chain on a large batch; "serve": the batched chain on the
few events a serving launch holds; "single": the per-event chain).

    python -m paper_1305_4855_amd.tune --config c3 --events 64                # batched chain
    python -m paper_1305_4855_amd.tune --config c3 --mode serve --events 4    # serving launches
    python -m paper_1305_4855_amd.tune --config c2 --mode single               # per-event chain
"""
from __future__ import annotations

import argparse
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")

SPACE = {
    "batch": dict(vote_cols=(16, 32, 64), vote_grid=(1024, 2048, 4096), peak_planes=(8, 16, 32),
                  assign_blocks=(32, 64, 128), prep_rows=(64, 128, 256), vote_threads=(512, 1024)),
    "serve": dict(vote_cols=(8, 16, 32), vote_grid=(512, 1024, 2048), peak_planes=(8, 16, 32),
                  assign_blocks=(64, 128, 256), prep_rows=(32, 64, 128, 256), vote_threads=(512, 1024)),
    "single": dict(vote_cols=(4, 8, 16, 32), peak_planes=(4, 8, 16), assign_blocks=(256, 512, 1024),
                   prep_rows=(16, 32, 64, 128, 256), vote_threads=(512, 1024)),
}
DEFAULT = dict(vote_threads=1024, vote_grid=0, peak_planes=8, vote_cols=0, assign_blocks=0, prep_rows=0)


def path_of(cfg, max_hits: int) -> str:
    """The kernel path a plan takes: window tables (at most 65535 hits, n_phi >= 128) or LDS slabs."""
    return "pt" if max_hits <= 65535 and cfg.n_phi >= 128 else "slab"


def cache_key(cfg, arch: str, max_hits: int, mode: str) -> str:
    return (f"{arch}:{cfg.n_phi}x{cfg.n_qpt}x{cfg.n_d0}:i{cfg.acc_bits}:f{cfg.frac_bits}:"
            f"{path_of(cfg, max_hits)}:{mode}")


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def apply(plan, mode: str = "batch") -> dict:
    """Set the cached tuning for this plan's grid, path and mode on this device, if there is one (a
    serving plan without its own entry takes the batch entry)."""
    cache = load_cache()
    arch = device_arch()
    entry = cache.get(cache_key(plan.cfg, arch, plan.max_hits, mode))
    if entry is None and mode == "serve":
        entry = cache.get(cache_key(plan.cfg, arch, plan.max_hits, "batch"))
    if entry:
        plan.set_tuning(**{**DEFAULT, **entry["best"]})
    return plan.tuning


def _digest(tensors, per_event: bool) -> tuple:
    """Position-weighted int64 sums (wrapping) of every output buffer (event by event for batch
    buffers, whose first dimension is the event)."""
    import torch
    out = []
    for t in tensors:
        if t is None:
            continue
        for chunk in (t if per_event else [t]):
            v = chunk.reshape(-1).to(torch.int64)
            w = torch.arange(v.numel(), device=v.device, dtype=torch.int64) % 1000003 + 1
            out.append(int((v * w).sum().item()))
    return tuple(out)


def _timed(run, reps: int) -> float:
    import torch
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        run()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(cfg, events, mode: str = "batch", reps: int = 3, passes: int = 2, log=print) -> dict:
    import torch

    from . import hough as H

    batched = mode in ("batch", "serve")
    max_hits = cfg.max_hits_per_event if batched else max(16384, max(e.n for e in events))
    plan = H.Plan(cfg, max_hits=max_hits)
    if batched:
        total = sum(e.n for e in events)
        bufs = H.BatchBuffers(plan, len(events), total, cap_peaks=1 << 21 if cfg.n_cot else 1 << 19,
                              cap_pairs=1 << 24)
        bufs.load(events)

        def run():
            bufs.run(cfg.threshold)

        def outputs():
            return (bufs.acc, bufs.peaks, bufs.offsets, bufs.hit_idx, bufs.status, bufs.zv)
    else:
        big = bool(cfg.n_cot)  # the large grid: about 1.5 M candidates and 16 M pairs per event
        bufs = H.EventBuffers(plan, cap_peaks=1 << 21 if big else 1 << 19, cap_pairs=1 << 25 if big else 1 << 24)
        x, y, lay, z = H.hits_to_device(events[0])
        hits = H.make_hits(x, y, lay, z)

        def run():
            bufs.run(hits, cfg.threshold)

        def outputs():
            return (bufs.acc, bufs.peaks, bufs.offsets, bufs.hit_idx, bufs.status, bufs.zv)
    space = SPACE[mode]
    if path_of(cfg, max_hits) == "pt":
        space = {k: v for k, v in space.items() if k != "vote_threads"}
    else:
        space = {k: v for k, v in space.items() if k not in ("vote_cols", "prep_rows")}
    seen = {}
    ref = None

    def measure(t: dict) -> float:
        nonlocal ref
        key = tuple(sorted(t.items()))
        if key in seen:
            return seen[key]
        plan.set_tuning(**t)
        run()
        torch.cuda.synchronize()
        flags = bufs.status.view(-1, H.STATUS_BYTES // 4)[:, 5].cpu().numpy()
        if flags.any():
            raise RuntimeError(f"capacity too small for the tuning events (flags {int(flags.max())})")
        d = _digest(outputs(), per_event=batched)
        if ref is None:
            ref = d
        elif d != ref:
            raise RuntimeError(f"results differ for tile shape {t}")
        ms = _timed(run, reps)
        seen[key] = ms
        log(f"  {t}: {ms:.4f} ms")
        return ms

    best = dict(DEFAULT)
    best_ms = measure(best)
    for _ in range(passes):
        for knob, values in space.items():
            for v in values:
                t = dict(best, **{knob: v})
                ms = measure(t)
                if ms < best_ms:
                    best, best_ms = t, ms
    table = sorted(({"ms": round(ms, 4), **dict(k)} for k, ms in seen.items()), key=lambda r: r["ms"])
    return dict(best=best, best_ms=round(best_ms, 4), mode=mode, n_events=len(events), max_hits=max_hits,
                table=table, when=time.strftime("%Y-%m-%d %H:%M:%S"))


def main() -> int:
    from . import configs, synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c3")
    ap.add_argument("--mode", choices=("batch", "serve", "single"), default="batch")
    ap.add_argument("--events", type=int, default=64)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--cache", default=CACHE, help="cache file to update (default: the package's)")
    args = ap.parse_args()
    cfg = configs.get(args.config)
    n = args.events if args.mode != "single" else 1
    events = [synth.make_event(cfg, i) for i in range(n)]
    arch = device_arch()
    print(f"tuning {cfg.name} ({args.mode}) on {arch} with {len(events)} events", flush=True)
    entry = tune(cfg, events, mode=args.mode, reps=args.reps, log=lambda s: print(s, flush=True))
    key = cache_key(cfg, arch, entry["max_hits"], args.mode)
    cache = {}
    if os.path.exists(args.cache):
        with open(args.cache) as f:
            cache = json.load(f)
    cache[key] = entry
    with open(args.cache, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    print(json.dumps({"key": key, "best": entry["best"], "best_ms": entry["best_ms"]}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
