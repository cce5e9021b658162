#!/usr/bin/env python3
"""Throughput of the Hough-transform hot path on one MI355X.

One step = one event through the whole path (prep -> vote -> peaks -> assign)
on the dense single-event workload: 1000 helical tracks (10 % displaced) plus
20 % noise hits, about 12k hits, voted into a 512 x 256 x 64 int32
phi0 x q/pT x d0 accumulator (32 MiB), candidates at >= 7 votes that are local
maxima of their 3x3x3 neighbourhood, and their CSR hit lists.  Inputs are
resident in HBM before the timed region; every step recomputes everything.

Prints one JSON line (see the keys below).  The `roofline` object is for the
dominant kernel of the step (the longer of the window-table vote and the
assignment, both HBM-bound), timed inside the timed region by HIP events that
the kernel's own launch records on the stream it runs on; `kernel_rooflines`
holds both.  `cpu_baseline` times the CPU oracle on the same event.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/s and hit-votes/s at 1 MI355X (batched vs plain), p99 event latency"
# MI355X: 256 CUs at 2.4 GHz; an LDS atomic of a 64-wide wave (ds_add_u32) issues once per 4 clocks per CU
# (16 lanes/clk/CU), so 256 * 2.4e9 * 16 = 9.83e12 atomic adds/s.  This unit-count figure is only the
# fallback: the micro-benchmarks measure the rate on the device and replace it.
CUS, CLOCK_HZ, LDS_ATOMIC_LANES_PER_CLK = 256, 2.4e9, 16
LDS_ATOMIC_PEAK_GVOTES = CUS * CLOCK_HZ * LDS_ATOMIC_LANES_PER_CLK / 1e9
VOTE_PAIR_PEAK_GOPS = LDS_ATOMIC_PEAK_GVOTES / 2
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c2.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1305_4855_amd", "csrc", "hough.hip")


def src_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def physical_cores() -> int:
    """Physical cores of the host (lscpu: distinct (core, socket) pairs); the logical CPU count
    when lscpu is not there."""
    try:
        out = subprocess.run(["lscpu", "-p=CORE,SOCKET"], capture_output=True, text=True, timeout=10).stdout
        pairs = {ln for ln in out.splitlines() if ln and not ln.startswith("#")}
        if pairs:
            return len(pairs)
    except (OSError, subprocess.SubprocessError):
        pass
    return os.cpu_count() or 1


def cpu_baseline(cfg, ev):
    """The oracle as it stands on the host cores: one full event of the dense workload (vote with
    OpenMP over d0 planes on every physical core, peaks and assign single-threaded), then the same
    event with one thread; and the oracle chain on the paper detector's curved events against the
    number of tracks."""
    from oracle import oracle as O
    O.build()
    g = O.Cfg(cfg)
    cores = physical_cores()
    runs = {}
    for threads in (cores, 1):
        used = O.set_threads(threads)
        t0 = time.perf_counter()
        acc, nv = O.vote(g, ev)
        n, pk = O.peaks(g, acc, cfg.threshold)
        O.assign(g, ev, pk)
        runs[used] = time.perf_counter() - t0
    O.set_threads(cores)
    dt = runs[max(runs)]
    # the same oracle chain on the paper detector's curved events against the number of tracks (the
    # quantity of the paper's CPU/GPU timing figure; the GPU side is in the quality section)
    from paper_1305_4855_amd import configs, synth
    vs_tracks = []
    for ntr in (50, 500, 2000, 4000):
        c7 = configs.C7.with_(n_tracks=ntr)
        e7 = synth.make_event(c7, 0)
        g7 = O.Cfg(c7)
        t1 = time.perf_counter()
        a7, _ = O.vote(g7, e7)
        n7, p7 = O.peaks(g7, a7, c7.threshold)
        O.assign(g7, e7, p7)
        vs_tracks.append({"tracks": ntr, "hits": e7.n, "oracle_ms_per_event": round((time.perf_counter() - t1) * 1e3, 2)})
    return {"value": round(1.0 / dt, 4), "unit": "events/s", "cores": max(runs), "kind": "oracle",
            "sample": (f"1 full event of the same workload ({ev.n} hits, {nv} hit-votes, {n} candidates): "
                       f"vote on {max(runs)} OpenMP threads (the host's physical cores), peaks and assign "
                       f"single-threaded; {dt:.1f} s"),
            "hit_votes_per_s": round(nv / dt, 1),
            "one_thread": {"value": round(1.0 / runs[1], 4), "unit": "events/s", "cores": 1,
                           "seconds": round(runs[1], 2)},
            "paper_detector_vs_tracks": vs_tracks}


def bench_roofline_probe():
    """The ceilings the roofline fractions are taken against, measured on this device by the
    micro-benchmarks of paper_1305_4855_amd/csrc/roofline_probe.hip: conflict-free LDS atomic adds
    (no return, the slab votes' operation), 32-bit LDS reads and writes at the same addresses as
    controls, 128-bit LDS reads (LDS bandwidth), and an HBM streaming copy and fill of 2 GiB."""
    from paper_1305_4855_amd import probe

    blocks = CUS * 4
    lds = {k: probe.lds(k, blocks) for k in ("atomic", "read32", "write32", "read128", "atomic_rtn", "vote_pair")}
    out = {}
    for k, r in lds.items():
        out[f"lds_{k}"] = {"lane_ops_per_s": round(r["lane_ops_per_s"], 1),
                           "lanes_per_clk_per_cu_at_2.4GHz": round(r["lane_ops_per_s"] / (CUS * CLOCK_HZ), 2),
                           "bytes_per_clk_per_cu_at_2.4GHz": round(r["bytes_per_s"] / (CUS * CLOCK_HZ), 1),
                           "us_per_launch": r["us_per_launch"], "workgroups": blocks}
    for k in ("copy", "fill"):
        r = probe.hbm(k)
        out[f"hbm_{k}"] = {"gb_per_s": r["gb_per_s"], "bytes": r["bytes"], "us_per_launch": r["us_per_launch"]}
    out["note"] = ("LDS rates of 1024-thread workgroups, 16 independent instructions per loop iteration; "
                   "the LDS-atomic rooflines use lds_atomic.lane_ops_per_s as their peak, the r-z vote's "
                   "lds_vote_pair.lane_ops_per_s (add-with-return plus restoring add)")
    return out


CHAIN_BYTES_NOTE = ("algorithmic HBM bytes of one pass of the chain: accumulator written by the vote and read by the "
                    "peak finder, 16-byte candidate rows written and read again by the assignment, 4-byte CSR "
                    "offsets and 4-byte hit indices written (hits and tables are cache-resident)")


def chain_hbm_bytes(acc_bytes: int, candidates: int, pairs: int, n_events: int) -> int:
    return 2 * acc_bytes + 32 * candidates + 4 * (candidates + n_events) + 4 * pairs


def assign_hbm_bytes(candidates: int, pairs: int) -> int:
    """Algorithmic bytes of one assignment launch: each candidate's 16-byte row read and its 4-byte
    CSR offset written, the closing offset, and one 4-byte hit index per (hit, candidate) pair."""
    return 20 * candidates + 4 + 4 * pairs


def bufs_max_pairs(st_i32: np.ndarray) -> int:
    return int(st_i32.view(np.int64)[:, 3].max()) if st_i32.shape[0] else 0


def check_flags(st_i32: np.ndarray, what: str) -> dict:
    """Per-event status flags of a batch (int32 view of the status rows): the OR of all flags and the
    number of events with any flag set.  Timed runs must not truncate work, so a set flag is an error."""
    fl = st_i32[:, 5]
    out = {"status_flags_or": int(np.bitwise_or.reduce(fl)) if fl.size else 0,
           "events_flagged": int(np.count_nonzero(fl))}
    if out["events_flagged"]:
        raise RuntimeError(f"{what}: {out['events_flagged']} events flagged (flags {out['status_flags_or']}): "
                           "candidate or pair capacity too small")
    return out


def sized_batch(H, torch, plan, events, threshold, stream, cap_peaks=1 << 18, cap_pairs=1 << 22):
    """Batch buffers whose per-event capacities hold the largest event's candidates and pairs: one
    sizing run, then buffers sized to the largest counts (rounded up to a power of two)."""
    total = sum(e.n for e in events)
    while True:
        bufs = H.BatchBuffers(plan, len(events), total, cap_peaks=cap_peaks, cap_pairs=cap_pairs)
        bufs.load(events)
        bufs.run(threshold, stream)
        torch.cuda.synchronize()
        st = bufs.status.cpu().numpy().view("int32")
        need_pk = int(st[:, 4].max()) if len(events) else 0
        need_pr = bufs_max_pairs(st)
        if need_pk <= cap_peaks and need_pr <= cap_pairs:
            return bufs, cap_peaks, cap_pairs
        del bufs
        torch.cuda.empty_cache()
        cap_peaks = max(cap_peaks, 1 << int(need_pk - 1).bit_length())
        cap_pairs = max(cap_pairs, 1 << int(need_pr - 1).bit_length())


def bench_batched(H, torch, n_events: int, reps: int):
    """The batched workload: n_events events with uneven hit counts (Gamma-Poisson track counts,
    mean 500, 5 % displaced, 20 % noise) on the same 512x256x64 int32 grid, in one persistent
    launch chain (and replayed as a hipGraph), against the plain per-event chain on the same
    events (all hits resident in HBM beforehand)."""
    from paper_1305_4855_amd import configs, synth, tune

    cfg = configs.C3
    events = [synth.make_event(cfg, i) for i in range(n_events)]
    plan = H.Plan(cfg, max_hits=cfg.max_hits_per_event)
    tuning = tune.apply(plan, "batch")
    total = sum(e.n for e in events)
    stream = torch.cuda.current_stream()
    bufs, cap_peaks, cap_pairs = sized_batch(H, torch, plan, events, cfg.threshold, stream)
    for _ in range(2):
        bufs.run(cfg.threshold, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        bufs.run(cfg.threshold, stream)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    st = bufs.status.cpu().numpy().view("int32")
    votes = int(bufs.status.cpu().numpy().view("int64")[:, 1].sum())
    peaks = int(st[:, 4].sum())
    pairs = int(st.view(np.int64)[:, 3].sum())
    flags = check_flags(st, "batched")
    # the persistent vote kernel of the batch, timed by its own start/end events
    vp = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in vp:
        a.record(stream)
        b.record(stream)
    torch.cuda.synchronize()
    for a, b in vp:
        plan.set_vote_events(a, b)
        bufs.run(cfg.threshold, stream)
    torch.cuda.synchronize()
    plan.set_vote_events(None, None)
    vote_batch_ms = sum(a.elapsed_time(b) for a, b in vp) / reps
    vote_bytes = n_events * plan.acc_bytes
    vote_gbs = vote_bytes / (vote_batch_ms * 1e-3) / 1e9
    chain_bytes = chain_hbm_bytes(n_events * plan.acc_bytes, peaks, pairs, n_events)
    # the same chain captured once in a hipGraph
    gstream = torch.cuda.Stream()
    graph = H.Graph(bufs, cfg.threshold, gstream)
    graph.launch(gstream)
    gstream.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.launch(gstream)
    gstream.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    graph.close()
    # plain per-event chain over the same events, with the single-event tuning of this grid
    plan_single = H.Plan(cfg, max_hits=cfg.max_hits_per_event)
    tune.apply(plan_single, "single")
    ev_bufs = H.EventBuffers(plan_single, cap_peaks=cap_peaks, cap_pairs=cap_pairs)
    dev_hits = []
    for e in events:
        x, y, lay, _ = H.hits_to_device(e)
        dev_hits.append((x, y, lay, H.make_hits(x, y, lay)))
    for h in dev_hits[:4]:
        ev_bufs.run(h[3], cfg.threshold, stream)
    torch.cuda.synchronize()
    plain_reps = max(1, reps // 2)
    t0 = time.perf_counter()
    for _ in range(plain_reps):
        for h in dev_hits:
            ev_bufs.run(h[3], cfg.threshold, stream)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / plain_reps
    check_flags(bufs.status.cpu().numpy().view("int32"), "batched (after the graph replays)")
    del bufs
    return {
        "workload": f"batch of {n_events} uneven events (c3): Gamma-Poisson tracks mean 500 in [50, 2000], "
                    f"5% displaced, 20% noise, 512x256x64 int32",
        "hits": total, "hits_min": min(e.n for e in events), "hits_max": max(e.n for e in events),
        "hit_votes": votes, "candidates": peaks, "pairs": pairs, "tuning": tuning,
        "cap_peaks": cap_peaks, "cap_pairs": cap_pairs, "max_candidates_per_event": int(st[:, 4].max()),
        "max_pairs_per_event": int(bufs_max_pairs(st)), **flags,
        "events_per_s_batched": round(n_events / t_batch, 2),
        "events_per_s_graph": round(n_events / t_graph, 2),
        "events_per_s_plain": round(n_events / t_plain, 2),
        "hit_votes_per_s_batched": round(votes / t_batch, 1),
        "speedup_batched_vs_plain": round(t_plain / t_batch, 3),
        "ms_per_batch": round(t_batch * 1e3, 4), "ms_per_batch_graph": round(t_graph * 1e3, 4),
        "ms_plain_all_events": round(t_plain * 1e3, 4),
        "roofline_vote": {"kernel": "k_vote_pt (persistent, whole batch)", "bound": "hbm",
                          "achieved": round(vote_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(vote_gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(vote_batch_ms, 4),
                          "bytes_per_launch": vote_bytes, "hit_votes_per_s": round(votes / (vote_batch_ms * 1e-3), 1),
                          "bytes_note": "every accumulator written once (the window-count tables it reads are "
                                        "cache-resident)"},
        "chain_hbm": {"bytes_per_batch": chain_bytes,
                      "achieved": round(chain_bytes / t_batch / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(chain_bytes / t_batch / 1e9 / HBM_PEAK_GBS, 4),
                      "bytes_note": CHAIN_BYTES_NOTE},
    }


def bench_large_grid(H, torch, reps: int):
    """The large-grid workload: 64 events of 600 prompt tracks plus two displaced vertices, 20 %
    noise, with z, on a 1024x512x128 int16 grid, batched, followed by the second-stage
    cot(theta) x z0 (128 x 128) vote of every candidate.  The r-z stage's share is the
    difference between the chain with and without it.  The vertex transform of all events'
    candidates (batched vote and peaks) is timed on its own."""
    from paper_1305_4855_amd import configs, synth, tune

    cfg = configs.C4
    events = [synth.make_event(cfg, i) for i in range(cfg.n_events)]
    plan = H.Plan(cfg, max_hits=cfg.max_hits_per_event)
    tuning = tune.apply(plan, "batch")
    total = sum(e.n for e in events)
    stream = torch.cuda.current_stream()
    bufs, cap_peaks, cap_pairs = sized_batch(H, torch, plan, events, cfg.threshold, stream, 1 << 20, 1 << 24)
    times = {}
    for with_z in (False, True):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            bufs.run(cfg.threshold, stream, zvote=with_z)
        b.record(stream)
        torch.cuda.synchronize()
        times[with_z] = a.elapsed_time(b) / reps
    # the plain per-event chain (prep, vote, peaks, assign, r-z stage) over the same events
    plan_single = H.Plan(cfg, max_hits=cfg.max_hits_per_event)
    tune.apply(plan_single, "single")  # the single-event tuning of this grid, if there is one
    ev_bufs = H.EventBuffers(plan_single, cap_peaks=cap_peaks, cap_pairs=cap_pairs)
    dev_hits = []
    for e in events:
        x, y, lay, z = H.hits_to_device(e)
        dev_hits.append((x, y, lay, z, H.make_hits(x, y, lay, z)))
    ev_bufs.run(dev_hits[0][4], cfg.threshold, stream)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for h in dev_hits:
        ev_bufs.run(h[4], cfg.threshold, stream)
    b.record(stream)
    torch.cuda.synchronize()
    plain_ms = a.elapsed_time(b)
    del ev_bufs, dev_hits, plan_single
    # the second transform (vertex space) of every event's candidates, batched
    vp = H.VertexPlan.of(plan)
    vb = H.VertexBatchBuffers(vp, len(events), cap_peaks, 1 << 16)
    vb.run(bufs.peaks, bufs.status, cfg.v_threshold, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        vb.run(bufs.peaks, bufs.status, cfg.v_threshold, stream)
    b.record(stream)
    torch.cuda.synchronize()
    vertex_ms = a.elapsed_time(b) / reps
    stv = vb.status.cpu().numpy()
    vertex_votes = int(stv.view("int64")[:, 1].sum())
    vertex_cands = int(stv[:, 4].sum())
    del vb
    st = bufs.status.cpu().numpy()
    votes = int(st.view("int64")[:, 1].sum())
    cands = int(st[:, 4].sum())
    pairs = int(st.view("int64")[:, 3].sum())
    flags = check_flags(st, "large grid")
    del bufs
    zv_ms = times[True] - times[False]
    # one (hit, cot(theta) row) evaluation of the r-z vote is an LDS add-with-return and, for a hit
    # that is not the first of its candidate in the z0 bin, the restoring add: the vote-pair
    # micro-benchmark measures exactly that pair
    zv_evals = pairs * cfg.n_cot
    zv_rate = zv_evals / (zv_ms * 1e-3) / 1e9
    pair_peak = VOTE_PAIR_PEAK_GOPS
    return {
        "workload": f"batch of {len(events)} events (c4): 600 prompt tracks + 2 displaced vertices, 20% noise, "
                    f"1024x512x128 int16, then 128x128 cot(theta) x z0 vote per candidate",
        "hits": total, "hit_votes": votes, "candidates": cands, "pairs": pairs, **flags, "tuning": tuning,
        "cap_peaks": cap_peaks, "cap_pairs": cap_pairs,
        "ms_per_batch": round(times[True], 3), "ms_per_batch_without_zvote": round(times[False], 3),
        "events_per_s": round(len(events) / times[True] * 1e3, 2),
        "events_per_s_without_zvote": round(len(events) / times[False] * 1e3, 2),
        "events_per_s_plain": round(len(events) / plain_ms * 1e3, 2),
        "speedup_batched_vs_plain": round(plain_ms / times[True], 3),
        "zvote_ms_per_event": round(zv_ms / len(events), 4),
        "roofline_zvote": {"kernel": "k_zvote", "bound": "lds_atomic", "achieved": round(zv_rate, 1),
                           "peak": round(pair_peak, 1), "unit": "G (hit, row) evaluations/s",
                           "frac": round(zv_rate / pair_peak, 4), "evaluations_per_batch": zv_evals,
                           "ms_per_batch": round(zv_ms, 3),
                           "peak_note": "LDS add-with-return plus restoring add per evaluation, as measured by "
                                        "the vote-pair micro-benchmark (unit-count fallback: half the LDS-atomic "
                                        "lane rate)"},
        "vertex_ms_per_batch": round(vertex_ms, 3), "vertex_ms_per_event": round(vertex_ms / len(events), 4),
        "vertex_votes": vertex_votes, "vertex_candidates": vertex_cands,
        "vertex_gvotes_per_s": round(vertex_votes / (vertex_ms * 1e-3) / 1e9, 1),
    }


def bench_small(H, torch, steps: int):
    """The small single event (c1: 10 prompt tracks, 256 x 256 phi0 x q/pT, threshold 8), plain
    chain per event: bound by launch latency, not by the GPU's throughput."""
    from paper_1305_4855_amd import configs, synth

    cfg = configs.C1
    ev = synth.make_event(cfg, 0)
    plan = H.Plan(cfg, max_hits=4096)
    bufs = H.EventBuffers(plan, cap_peaks=1 << 14, cap_pairs=1 << 16)
    x, y, lay, _ = H.hits_to_device(ev)
    hits = H.make_hits(x, y, lay)
    stream = torch.cuda.current_stream()
    for _ in range(20):
        bufs.run(hits, cfg.threshold, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bufs.run(hits, cfg.threshold, stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st = H.status_dict(bufs.status)
    if st["flags"]:
        raise RuntimeError(f"small event: status flags {st['flags']}")
    return {"workload": "single small event (c1): 10 prompt tracks, 100 hits, 256x256 int32, threshold 8",
            "hits": ev.n, "hit_votes": st["n_votes"], "candidates": st["n_peaks"], "pairs": st["n_pairs"],
            "events_per_s": round(1.0 / dt, 1), "us_per_event": round(dt * 1e6, 2),
            "hit_votes_per_s": round(st["n_votes"] / dt, 1),
            "note": "prep, vote, peaks and assign launched per event; bound by launch latency"}


def bench_vertex(H, torch, reps: int):
    """The second transform (vertex space of the candidates) on one large-grid event: the event's
    first stage (prep, vote, peaks) gives its candidate list on the device; every candidate
    (votes >= the first-stage threshold) votes into 64 radius rows x 512 azimuth bins; then the
    vertex peaks.  The first stage of the same event is timed beside it (the paper counts the
    second transform as a second cost of the same kind)."""
    from paper_1305_4855_amd import configs, synth

    cfg = configs.C4
    ev = synth.make_event(cfg, 0)
    plan = H.Plan(cfg, max_hits=cfg.max_hits_per_event)
    bufs = H.EventBuffers(plan, cap_peaks=1 << 21, cap_pairs=1 << 20)
    x, y, lay, _ = H.hits_to_device(ev)
    hits = H.make_hits(x, y, lay)
    vp = H.VertexPlan.of(plan)
    vb = H.VertexBuffers(vp, cap_peaks=1 << 21, cap_vpeaks=1 << 16)
    stream = torch.cuda.current_stream()
    bufs.run(hits, cfg.threshold, stream, do_assign=False)
    vb.run(bufs.peaks, bufs.status, cfg.v_threshold, stream)
    torch.cuda.synchronize()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    first_ms = timed(lambda: bufs.run(hits, cfg.threshold, stream, do_assign=False))
    vote_ms = timed(lambda: H.vertex_vote(vp, bufs.peaks, bufs.status, vb.acc, vb.ws_vote, vb.status, stream))
    peaks_ms = timed(lambda: H.vertex_peaks(vp, vb.acc, cfg.v_threshold, vb.peaks, vb.ws_peaks, vb.status, stream))
    st1 = H.status_dict(bufs.status)
    stv = H.status_dict(vb.status)
    votes = stv["n_votes"]
    achieved = votes / (vote_ms * 1e-3) / 1e9
    peak = LDS_ATOMIC_PEAK_GVOTES  # one LDS atomic add per vertex vote
    return {
        "workload": "vertex space of one large-grid event (c4 event 0): every first-stage candidate votes into "
                    f"{cfg.n_vr} radius rows x {cfg.n_vphi} azimuth bins over [{cfg.vr_min}, {cfg.vr_max}) cm, "
                    f"then vertex peaks (threshold {cfg.v_threshold})",
        "hits": ev.n, "candidates": st1["n_peaks"], "vertex_votes": votes, "vertex_candidates": stv["n_peaks"],
        "groups": vp.groups, "first_stage_ms": round(first_ms, 4), "vertex_vote_ms": round(vote_ms, 4),
        "vertex_peaks_ms": round(peaks_ms, 4), "second_over_first": round((vote_ms + peaks_ms) / first_ms, 3),
        "roofline": {"kernel": "k_vvote + k_vreduce", "bound": "lds_atomic", "achieved": round(achieved, 1),
                     "peak": round(peak, 1), "unit": "Gvote/s (LDS atomic adds)", "frac": round(achieved / peak, 4),
                     "traffic": None},
        "note": "per-call time of back-to-back calls; the vote time includes the reduction of the partial "
                "vertex spaces (split in the kernel trace)",
    }


REFINE_WINDOW = 16      # 1/8 of a phi0 bin (frac_bits 7)
REFINE_MIN_LAYERS = 8   # of the ten layers


def bench_quality(H, torch):
    """Track-finding quality on the paper's own detector (layers at 11..110 cm, 0.4 mm x/y smear):
    the 50-straight-line example and curved prompt tracks at several track counts.  GPU chain
    outputs against the generator's truth, by hit share (a candidate is a track when 75 % of its
    list comes from it) and in parameter space (a candidate within one bin of a track's true bin);
    with the plain chain's time per event at each track count."""
    from paper_1305_4855_amd import configs, quality, synth

    out = []
    for base, ntr in ((configs.C6, 50), (configs.C7, 50), (configs.C7, 500), (configs.C7, 2000),
                      (configs.C7, 4000)):
        cfg = base.with_(n_tracks=ntr)
        ev = synth.make_event(cfg, 0)
        plan = H.Plan(cfg, max_hits=max(ev.n, 1))
        bufs = H.EventBuffers(plan, cap_peaks=1 << 18, cap_pairs=1 << 23)
        x, y, lay, _ = H.hits_to_device(ev)
        hits = H.make_hits(x, y, lay)
        bufs.run(hits, cfg.threshold)
        torch.cuda.synchronize()
        r = bufs.results()
        # time per event of the plain chain (prep, vote, peaks, assign) against the number of tracks,
        # the quantity of the paper's timing figure
        stream = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(20):
            bufs.run(hits, cfg.threshold, stream)
        b.record(stream)
        torch.cuda.synchronize()
        chain_ms = a.elapsed_time(b) / 20
        share = quality.quality(r["offsets"], r["hit_idx"], ev.track_id, ntr, cfg.threshold)
        param = quality.quality_params(cfg, ev.truth, ev.track_id, r["peaks"], cfg.threshold)
        # background suppression inside the bin: one hit per layer from the densest window of the
        # angle inside the bin (1/8 of a bin); candidates keeping >= 8 of the 10 layers
        n_c = r["peaks"].shape[0]
        out_h = torch.empty((max(n_c, 1), cfg.n_layers), dtype=torch.int32, device="cuda")
        out_l = torch.empty(max(n_c, 1), dtype=torch.int32, device="cuda")
        H.refine(plan, bufs.peaks[: max(n_c, 1)], bufs.offsets, bufs.hit_idx, bufs.ws, bufs.status,
                 REFINE_WINDOW, out_h, out_l)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(5):
            H.refine(plan, bufs.peaks[: max(n_c, 1)], bufs.offsets, bufs.hit_idx, bufs.ws, bufs.status,
                     REFINE_WINDOW, out_h, out_l)
        b.record(stream)
        torch.cuda.synchronize()
        refine_ms = a.elapsed_time(b) / 5
        ro, rh, kept = quality.refined_csr(out_h[:n_c].cpu().numpy(), out_l[:n_c].cpu().numpy(), REFINE_MIN_LAYERS)
        share_r = quality.quality(ro, rh, ev.track_id, ntr, cfg.threshold)
        param_r = quality.quality_params(cfg, ev.truth, ev.track_id, r["peaks"][kept], cfg.threshold)
        out.append({"workload": cfg.name, "tracks": ntr, "hits": ev.n,
                    "grid": f"{cfg.n_phi}x{cfg.n_qpt}x{cfg.n_d0}", "threshold": cfg.threshold,
                    "candidates": r["status"]["n_peaks"], "chain_ms_per_event": round(chain_ms, 4),
                    "hit_share": {k: share[k] for k in ("efficiency", "purity", "duplicates_per_found_track")},
                    "parameter_space": {k: param[k] for k in ("efficiency", "purity")},
                    "suppressed": {"window": REFINE_WINDOW, "min_layers": REFINE_MIN_LAYERS,
                                   "candidates": int(kept.size), "refine_ms": round(refine_ms, 4),
                                   "hit_share": {k: share_r[k] for k in ("efficiency", "purity",
                                                                         "duplicates_per_found_track")},
                                   "parameter_space": {k: param_r[k] for k in ("efficiency", "purity")}}})
        del bufs, plan
    return {"note": "context, not a parity figure: the paper quotes about 80 % efficiency at a few thousand "
                    "tracks and 86 % for curved prompt tracks, with comparable purity, on its own simulation",
            "runs": out}


# VALU lane-instructions per sample of k_vote_cr (SQ_INSTS_VALU x 64 / samples, counted on the
# kernel as built: 7.9e7 wave instructions for 1.024e7 samples), and the chip's 32-bit VALU issue
# rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
CR_VALU_PER_SAMPLE = 495
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12


def bench_cr(H, torch, reps: int):
    """The vote with each hit's own radius on the paper's detector (x/y smear): 4000 curved prompt
    tracks (40 000 hits) on the 256 x 256 phi0 x q/pT grid, every sample computed (integer
    arcsine); then the unchanged peak finder."""
    from paper_1305_4855_amd import configs, synth

    cfg = configs.C7.with_(n_tracks=4000)
    ev = synth.make_event(cfg, 0)
    plan = H.Plan(cfg, max_hits=ev.n)
    acc = torch.empty((cfg.n_d0, cfg.n_qpt, cfg.n_phi), dtype=torch.int32, device="cuda")
    st = torch.zeros(H.STATUS_BYTES // 4, dtype=torch.int32, device="cuda")
    ws = torch.empty(plan.ws_bytes(1 << 16), dtype=torch.uint8, device="cuda")
    pk = torch.empty((1 << 16, 4), dtype=torch.int32, device="cuda")
    x, y, lay, _ = H.hits_to_device(ev)
    hits = H.make_hits(x, y, lay)
    stream = torch.cuda.current_stream()
    H.vote_cr(plan, hits, acc, st, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        H.vote_cr(plan, hits, acc, st, stream)
    b.record(stream)
    torch.cuda.synchronize()
    vote_ms = a.elapsed_time(b) / reps
    H.peaks(plan, acc, cfg.threshold, pk, ws, st, stream)
    torch.cuda.synchronize()
    s = H.status_dict(st)
    samples = ev.n * cfg.n_qpt * cfg.n_d0
    return {"workload": "paper detector (layers 11..110 cm, 0.4 mm x/y smear), 4000 curved prompt tracks, "
                        "256x256 phi0 x q/pT, per-hit radius with integer arcsine",
            "hits": ev.n, "samples": samples, "votes": s["n_votes"], "candidates": s["n_peaks"],
            "vote_ms": round(vote_ms, 4), "samples_per_s": round(samples / (vote_ms * 1e-3), 1),
            "roofline": {"kernel": "k_vote_cr", "bound": "alu",
                         "achieved": round(samples * CR_VALU_PER_SAMPLE / (vote_ms * 1e-3) / 1e12, 3),
                         "peak": VALU_PEAK_T, "unit": "T VALU lane-instructions/s",
                         "frac": round(samples * CR_VALU_PER_SAMPLE / (vote_ms * 1e-3) / 1e12 / VALU_PEAK_T, 4),
                         "traffic": None, "valu_per_sample": CR_VALU_PER_SAMPLE},
            "note": "ALU-bound: a 30-step CORDIC, an integer square root and a double division per sample; "
                    "VALU instructions per sample from SQ_INSTS_VALU of this kernel"}


def bench_serving(H, torch, runs, pool_size: int = 256):
    """Streaming trigger serving: for each (rate_hz, duration_s) of `runs`, Poisson arrivals at that
    rate, event sizes as in the batched workload, admitted into device-resident slots within a
    64 GiB accumulator budget, continuous batching over concurrent lanes (see
    paper_1305_4855_amd/serve.py).  One server (slots allocated once) serves every run."""
    from paper_1305_4855_amd import configs, serve, synth, tune

    cfg = configs.C5
    pool = [synth.make_event(cfg, i) for i in range(pool_size)]
    plan = H.Plan(cfg, max_hits=cfg.max_hits_per_event)
    tuning = tune.apply(plan, "serve")  # tuned on launches of a few events, as serving makes them
    # per-event capacities hold the pool's largest event (2000 tracks: about 2.4e5 candidates and
    # 1.3e7 hit-candidate pairs), so no served list is cut
    srv = serve.Server(plan, cfg.threshold, budget_bytes=cfg.hbm_budget_bytes, n_contexts=4, max_batch=64,
                       cap_peaks=1 << 19, cap_pairs=1 << 24, hits_per_event=8192, topk=64)
    # warm up every context once
    warm = np.linspace(0.0, 0.01, 4 * srv.max_batch)
    srv.serve(pool, warm, np.arange(len(warm)) % pool_size)
    results = []
    for i, (rate_hz, duration_s) in enumerate(runs):
        arrivals = serve.poisson_arrivals(rate_hz, duration_s, seed=13054855 + i)
        rng = np.random.default_rng([13054855, 5, 1 + i])
        pool_idx = rng.integers(0, pool_size, size=len(arrivals))
        print(f"[bench] serving {len(arrivals)} arrivals at {rate_hz:.0f} Hz over {duration_s:.0f} s in "
              f"{srv.n_slots} slots", file=sys.stderr, flush=True)
        stats = srv.serve(pool, arrivals, pool_idx, progress=lambda t, n, q: print(
            f"[bench] serving t={t:.0f}s served={n} queued={q}", file=sys.stderr, flush=True))
        if stats["events_flagged"]:
            raise RuntimeError(f"serving: {stats['events_flagged']} events flagged (flags {stats['status_flags_or']})")
        stats.update(tuning=tuning,
                     workload=f"Poisson arrivals at {rate_hz:.0f} Hz for {duration_s:.0f} s, sizes as the batched "
                              f"workload (pool of {pool_size} distinct events), 64 GiB device budget "
                              f"({srv.n_slots} resident slots, {len(srv.contexts)} launch contexts of up to "
                              f"{srv.max_batch} events), 512x256x64 int32",
                     latency_definition="arrival -> candidate list and hit lists complete in the event's device "
                                        "slot, status and first 64 candidates on the host")
        results.append(stats)
    return results


def bench_plain(H, torch, args):
    """The dense single event (c2), one event per launch chain: prep -> vote -> peaks -> assign."""
    from paper_1305_4855_amd import configs, synth, tune

    cfg = configs.C2
    ev = synth.make_event(cfg, 0)
    plan = H.Plan(cfg, max_hits=16384)
    tuning = tune.apply(plan, "single")
    bufs = H.EventBuffers(plan, cap_peaks=1 << 19, cap_pairs=1 << 24)
    x, y, lay, _ = H.hits_to_device(ev)
    hits = H.make_hits(x, y, lay)
    stream = torch.cuda.current_stream()

    if args.pmc_calibration:
        a = torch.empty(64 << 20, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    def step():
        H.prep(plan, hits, None, bufs.ws, bufs.status, stream)
        H.vote_prepared(plan, bufs.acc, bufs.ws, bufs.status, stream)
        H.peaks(plan, bufs.acc, cfg.threshold, bufs.peaks, bufs.ws, bufs.status, stream)
        H.assign(plan, bufs.peaks, bufs.offsets, bufs.hit_idx, bufs.ws, bufs.status, stream)

    for _ in range(args.warmup):
        step()
    # kernel durations: in a second pass of K steps, the vote and assignment kernels of every step
    # record their own start and end (kernel-accurate HIP events, recorded by the kernel's own
    # dispatch); the events are created beforehand
    def event_pairs():
        ps = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        for a, b in ps:
            a.record(stream)
            b.record(stream)
        return ps
    vpairs, apairs = event_pairs(), event_pairs()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the same K steps again with the two kernels recording their own start and end (the events
    # cost the stream a few microseconds per step, so the throughput comes from the pass above)
    for i in range(args.steps):
        plan.set_vote_events(*vpairs[i])
        plan.set_assign_events(*apairs[i])
        step()
    torch.cuda.synchronize()
    plan.set_vote_events(None, None)
    plan.set_assign_events(None, None)
    vote_kernel_ms = sum(a.elapsed_time(b) for a, b in vpairs) / args.steps
    assign_kernel_ms = sum(a.elapsed_time(b) for a, b in apairs) / args.steps

    # Per-stage launch durations: each stage launched `reps` times back to back on the same stream
    # between two HIP events (every stage is idempotent on the event's buffers), so the average is
    # the kernel time plus the launch gap, as a kernel trace reports it.
    reps = max(20, args.steps // 5)
    stage_calls = [
        lambda: H.prep(plan, hits, None, bufs.ws, bufs.status, stream),
        lambda: H.vote_prepared(plan, bufs.acc, bufs.ws, bufs.status, stream),
        lambda: H.peaks(plan, bufs.acc, cfg.threshold, bufs.peaks, bufs.ws, bufs.status, stream),
        lambda: H.assign(plan, bufs.peaks, bufs.offsets, bufs.hit_idx, bufs.ws, bufs.status, stream),
    ]
    stage_ms = []
    for call in stage_calls:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            call()
        b.record(stream)
        torch.cuda.synchronize()
        stage_ms.append(a.elapsed_time(b) / reps)
    vote_ms = vote_kernel_ms
    st = H.status_dict(bufs.status)

    # Track fit of every candidate (the next step after the assignment, outside the timed chain):
    # launched `reps` times back to back.  The fit is bound by its IEEE double arithmetic (the
    # moments are summed in double, in list order): 16 flops per list entry (three products and
    # three additions for the squares and cross term, eight moment updates with two more
    # products) and about 60 per candidate for the 3x3 solve; HBM bytes (lists, offsets, rows)
    # are reported beside it
    H.assign(plan, bufs.peaks, bufs.offsets, bufs.hit_idx, bufs.ws, bufs.status, stream)
    bufs.run_fit(hits, stream)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        bufs.run_fit(hits, stream)
    b.record(stream)
    torch.cuda.synchronize()
    fit_ms = a.elapsed_time(b) / reps
    n_fit = min(st["n_peaks"], bufs.peaks.shape[0])
    fit_bytes = 4 * st["n_pairs"] + 4 * (n_fit + 1) + 32 * n_fit + 8 * ev.n
    fit_gbs = fit_bytes / (fit_ms * 1e-3) / 1e9
    fit_flops = 16 * st["n_pairs"] + 60 * n_fit
    fit_tf = fit_flops / (fit_ms * 1e-3) / 1e12
    fit = {"workload": "algebraic circle fit of every candidate of the dense event (c2)",
           "candidates": n_fit, "pairs": st["n_pairs"], "ms_per_launch": round(fit_ms, 5),
           "candidates_per_s": round(n_fit / (fit_ms * 1e-3), 1),
           "roofline": {"kernel": "k_fit_res", "bound": "alu", "achieved": round(fit_tf, 3), "peak": 78.6,
                        "unit": "TFLOP/s (fp64)", "frac": round(fit_tf / 78.6, 4), "traffic": None,
                        "flops_per_launch": fit_flops},
           "hbm": {"bytes_per_launch": fit_bytes, "achieved_gbs": round(fit_gbs, 1),
                   "frac_of_8000": round(fit_gbs / 8000.0, 4)},
           "note": "per-launch time of back-to-back launches (kernel plus launch gap)"}

    if st["flags"]:
        raise RuntimeError(f"plain chain: status flags {st['flags']} (candidate or pair capacity too small)")
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    events_per_s = 1e3 / ms_per_step
    traffic = {}
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_src_sha256_16") == src_hash():
            traffic = {k: v["hbm_bytes_per_launch"] for k, v in tr["kernels"].items()}
    n_peaks = min(st["n_peaks"], bufs.peaks.shape[0])
    vote_bytes = plan.acc_bytes
    assign_bytes = assign_hbm_bytes(n_peaks, st["n_pairs"])

    def hbm_roofline(kernel, nbytes, ms, note):
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {"kernel": kernel, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic.get(kernel),
                "avg_launch_ms": round(ms, 5), "bytes_per_launch": nbytes, "bytes_note": note}
    kr = {
        "k_vote_pt": hbm_roofline("k_vote_pt", vote_bytes, vote_ms,
                                  "the 32 MiB accumulator written once; the window-count tables it reads "
                                  "(about 1.3 MB) are cache-resident"),
        "k_assign_pt": hbm_roofline("k_assign_pt", assign_bytes, assign_kernel_ms,
                                    "20 bytes per candidate (16-byte row read, 4-byte CSR offset written) plus "
                                    "4 bytes per (hit, candidate) pair written"),
    }
    dominant = max(kr.values(), key=lambda r: r["avg_launch_ms"])
    chain_bytes = chain_hbm_bytes(plan.acc_bytes, n_peaks, st["n_pairs"], 1)
    out = {
        "metric": METRIC,
        "value": round(events_per_s, 2),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "dense single event, 3-D displaced search (c2)", "mode": "plain",
                   "tracks": 1000, "noise_frac": 0.2, "displaced_frac": 0.1, "hits": ev.n,
                   "grid": [cfg.n_phi, cfg.n_qpt, cfg.n_d0], "acc": "int32", "threshold": cfg.threshold},
        "hit_votes_per_s": round(st["n_votes"] * events_per_s, 1),
        "tuning": tuning,
        "per_event": {"hit_votes": st["n_votes"], "candidates": st["n_peaks"], "pairs": st["n_pairs"],
                      "bad_hits": st["n_bad_hits"]},
        "stages_ms": {k: round(v, 5) for k, v in zip(("prep", "vote", "peaks", "assign"), stage_ms)},
        "stages_note": "each stage launched back to back, per-launch time including launch gaps",
        "roofline": dominant,
        "kernel_rooflines": kr,
        "vote_hit_votes_per_s": round(st["n_votes"] / (vote_ms * 1e-3), 1),
        "chain_hbm": {"bytes_per_step": chain_bytes, "achieved": round(chain_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                      "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(chain_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "bytes_note": CHAIN_BYTES_NOTE},
        "fit": fit,
    }
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline-probe", action="store_true",
                    help="skip the LDS/HBM micro-benchmarks (the LDS-atomic peak then falls back to unit counts)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-events", type=int, default=256)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the single-event section (profiling runs)")
    ap.add_argument("--no-small", action="store_true", help="skip the small-event section (profiling runs)")
    ap.add_argument("--no-large-grid", action="store_true")
    ap.add_argument("--no-vertex", action="store_true")
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--no-cr", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=20000.0)
    ap.add_argument("--serve-rate-low", type=float, default=14000.0,
                    help="a second, short serving run at this rate (0: none)")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        return 2

    import torch

    from paper_1305_4855_amd import hough as H

    torch.cuda.set_device(0)
    from paper_1305_4855_amd import configs, synth
    out = {"metric": METRIC, "value": None, "unit": "events/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int32", "data": "synthetic"}
    probe_res = None
    if not args.no_roofline_probe:
        global LDS_ATOMIC_PEAK_GVOTES, VOTE_PAIR_PEAK_GOPS
        probe_res = bench_roofline_probe()
        LDS_ATOMIC_PEAK_GVOTES = probe_res["lds_atomic"]["lane_ops_per_s"] / 1e9
        VOTE_PAIR_PEAK_GOPS = probe_res["lds_vote_pair"]["lane_ops_per_s"] / 1e9
        torch.cuda.empty_cache()
    if not args.no_plain:
        out = bench_plain(H, torch, args)
        torch.cuda.empty_cache()
    if not args.no_plain and not args.no_small:
        out["small_event"] = bench_small(H, torch, steps=500)
    if not args.no_batched:
        out["batched"] = bench_batched(H, torch, args.batch_events, reps=10)
    if not args.no_large_grid:
        out["large_grid"] = bench_large_grid(H, torch, reps=3)
    if not args.no_vertex:
        torch.cuda.empty_cache()
        out["vertex"] = bench_vertex(H, torch, reps=20)
    if not args.no_quality:
        out["quality"] = bench_quality(H, torch)
    if not args.no_cr:
        out["per_hit_radius"] = bench_cr(H, torch, reps=5)
    if not args.no_serving:
        torch.cuda.empty_cache()
        runs = [(args.serve_rate, args.serve_seconds)]
        if args.serve_rate_low > 0:
            runs.append((args.serve_rate_low, min(args.serve_seconds, 10.0)))
        res = bench_serving(H, torch, runs)
        out["serving"] = res[0]
        if len(res) > 1:
            out["serving_below_capacity"] = res[1]
    if probe_res is not None:
        out["roofline_probe"] = probe_res
    # the paper's own GPU figure, as context (its timing plots are not recoverable; only the prose survives)
    out["paper_context"] = {
        "gpu_hough_time_per_event": "several tens of ms per event of up to 5000 hits, data resident on the GPU, "
                                    "transfers excluded (Tesla C2075 / K20c; Sec. Preliminary Results)",
        "gpu_hough_events_per_s_implied": "a few tens per second",
        "cpu_openmp_speedup": "2.6 to 3.6 times one thread on a 4-core Ivy Bridge (Sec. Preliminary Results)",
        "note": "two-parameter transform on the paper's own simulation; not the workload measured here",
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(configs.C2, synth.make_event(configs.C2, 0))
    print(json.dumps(out, default=lambda o: o.item() if isinstance(o, np.generic) else str(o)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
