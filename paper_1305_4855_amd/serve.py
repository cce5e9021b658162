"""Trigger-style serving loop with continuous batching.

Events arrive as a Poisson process.  Admission is bounded by an accumulator
budget in device memory: the budget divided by one event's accumulator gives
the number of resident slots, each holding an accumulator together with that
event's workspace, candidate list and CSR hit list (allocated once, reused
without reallocation).  Slots are grouped into lanes; each lane owns a stream,
pinned host staging buffers and one batched launch chain (`hough_run_batch`).
Whenever a lane is free, the events that have arrived and are not yet admitted
are admitted into it, oldest first, as many as its slots and its packed hit
buffer hold: their hits are staged in pinned host memory and copied to the
device on the lane's stream, the batched chain runs, and the per-event status
plus the first `topk` candidates (in linear-index order) come back to pinned
host memory.  Lanes run concurrently, so events copied in on one lane overlap
the compute of another and the copy-out of a third (the event pipelining the
paper proposes for its throughput figure, Sec. "Preliminary Results").

Latency of an event = time from its arrival to the moment its candidate list
and hit lists are complete in device memory and its status and first
candidates are on the host.  The full lists stay resident until the slot is
reused (`on_complete` sees them): a flooded event has ~2e5 candidates, and
copying every list back at the offered rate would exceed the host link.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np
import torch

from . import hough as H


@dataclasses.dataclass
class Lane:
    idx: int
    bufs: H.BatchBuffers
    stream: torch.cuda.Stream
    done: torch.cuda.Event
    x_h: torch.Tensor
    y_h: torch.Tensor
    lay_h: torch.Tensor
    off_h: torch.Tensor
    status_h: torch.Tensor
    top_h: torch.Tensor
    busy: bool = False
    ids: Optional[np.ndarray] = None
    t_launch: float = 0.0


def slot_bytes(plan: H.Plan, cap_peaks: int, cap_pairs: int) -> int:
    """Device bytes one resident event occupies (accumulator, workspace, outputs, status)."""
    return (plan.acc_bytes + plan.ws_bytes(cap_peaks) + cap_peaks * 16 + (cap_peaks + 1) * 4 + cap_pairs * 4 +
            H.STATUS_BYTES)


class Server:
    """Continuous-batching server over `acc_budget_bytes // plan.acc_bytes` resident slots split into
    at most `max_lanes` lanes of at most `max_lane_events` slots each."""

    def __init__(self, plan: H.Plan, threshold: int, acc_budget_bytes: int, max_lanes: int = 4,
                 max_lane_events: int = 512, cap_peaks: int = 1 << 19, cap_pairs: int = 1 << 23,
                 hits_per_slot: int = 8192, topk: int = 64):
        self.plan, self.threshold, self.topk = plan, int(threshold), int(topk)
        self.cap_peaks, self.cap_pairs = int(cap_peaks), int(cap_pairs)
        slots = int(acc_budget_bytes // plan.acc_bytes)
        if slots < 1:
            raise ValueError("accumulator budget below one event's accumulator")
        n_lanes = max(1, min(int(max_lanes), slots))
        lane_events = max(1, min(int(max_lane_events), slots // n_lanes))
        self.slot_bytes, self.lane_events, self.n_lanes = slot_bytes(plan, cap_peaks, cap_pairs), lane_events, n_lanes
        # packed hit buffer of a lane: room for the largest event even if the lane holds one slot
        self.max_total_hits = max(lane_events * int(hits_per_slot), plan.max_hits)
        self.lanes: List[Lane] = []
        for i in range(n_lanes):
            bufs = H.BatchBuffers(plan, lane_events, self.max_total_hits, cap_peaks, cap_pairs)
            n = self.max_total_hits
            self.lanes.append(Lane(
                idx=i, bufs=bufs, stream=torch.cuda.Stream(), done=torch.cuda.Event(),
                x_h=torch.empty(n, dtype=torch.float32, pin_memory=True),
                y_h=torch.empty(n, dtype=torch.float32, pin_memory=True),
                lay_h=torch.empty(n, dtype=torch.uint8, pin_memory=True),
                off_h=torch.empty(lane_events + 1, dtype=torch.int32, pin_memory=True),
                status_h=torch.empty((lane_events, H.STATUS_BYTES // 4), dtype=torch.int32, pin_memory=True),
                top_h=torch.empty((lane_events, max(1, topk), H.PEAK_INTS), dtype=torch.int32, pin_memory=True)))

    @property
    def slots(self) -> int:
        return self.n_lanes * self.lane_events

    # ------------------------------------------------------------------ one lane
    def _launch(self, lane: Lane, ids: np.ndarray, pool_ids: np.ndarray, pool, now: float) -> None:
        evs = [pool[i] for i in pool_ids]
        sizes = np.fromiter((e.n for e in evs), dtype=np.int64, count=len(evs))
        offs = np.zeros(len(evs) + 1, dtype=np.int32)
        np.cumsum(sizes, out=offs[1:])
        n = int(offs[-1])
        if n > self.max_total_hits:
            raise RuntimeError("admitted events exceed the lane's hit buffer")
        if n:
            lane.x_h.numpy()[:n] = np.concatenate([e.x for e in evs])
            lane.y_h.numpy()[:n] = np.concatenate([e.y for e in evs])
            lane.lay_h.numpy()[:n] = np.concatenate([e.layer for e in evs])
        lane.off_h.numpy()[: len(evs) + 1] = offs
        b = lane.bufs
        m = len(evs)
        with torch.cuda.stream(lane.stream):
            if n:
                b.x[:n].copy_(lane.x_h[:n], non_blocking=True)
                b.y[:n].copy_(lane.y_h[:n], non_blocking=True)
                b.layer[:n].copy_(lane.lay_h[:n], non_blocking=True)
            b.hit_offsets[: m + 1].copy_(lane.off_h[: m + 1], non_blocking=True)
            b.run(self.threshold, lane.stream, n_events=m)
            lane.status_h[:m].copy_(b.status[:m], non_blocking=True)
            if self.topk:
                lane.top_h[:m].copy_(b.peaks[:m, : self.topk], non_blocking=True)
            lane.done.record(lane.stream)
        lane.busy, lane.ids, lane.t_launch = True, ids, now

    # ------------------------------------------------------------------ the loop
    def serve(self, pool, arrival_s: np.ndarray, pool_idx: np.ndarray,
              on_complete: Optional[Callable[[Lane, np.ndarray, np.ndarray], None]] = None,
              progress: Optional[Callable[[float, int, int], None]] = None, progress_every_s: float = 10.0) -> Dict:
        """Serve events arriving at `arrival_s` (seconds from the start, increasing), each a copy of
        `pool[pool_idx[i]]`.  Paced in wall-clock time.  Returns latency and throughput figures.
        `on_complete(lane, ids, pool_ids)` runs when a lane's batch is done, before the lane is reused;
        `progress(t, served, queued)` runs every `progress_every_s` seconds."""
        N = len(arrival_s)
        sizes = np.fromiter((e.n for e in pool), dtype=np.int64, count=len(pool))
        done_t = np.full(N, np.nan)
        flags_or = 0
        votes = 0
        candidates = 0
        pending: collections.deque = collections.deque()
        nxt = 0
        served = 0
        batch_sizes = []
        max_batch_hits = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        next_report = progress_every_s
        while served < N:
            now = time.perf_counter() - t0
            if progress is not None and now >= next_report:
                progress(now, served, len(pending))
                next_report += progress_every_s
            if nxt < N and arrival_s[nxt] <= now:
                k = int(np.searchsorted(arrival_s, now, side="right"))
                pending.extend(range(nxt, k))
                nxt = k
            progressed = False
            for lane in self.lanes:
                if lane.busy and lane.done.query():
                    tdone = time.perf_counter() - t0
                    m = len(lane.ids)
                    st = lane.status_h[:m].numpy()
                    done_t[lane.ids] = tdone
                    votes += int(st.view(np.int64)[:, 1].sum())
                    candidates += int(st[:, 4].sum())
                    flags_or |= int(np.bitwise_or.reduce(st[:, 5])) if m else 0
                    if on_complete is not None:
                        on_complete(lane, lane.ids, pool_idx[lane.ids])
                    served += m
                    lane.busy = False
                    progressed = True
            for lane in self.lanes:
                if not lane.busy and pending:
                    # oldest first, as many as the lane's slots and hit buffer hold
                    ids_l, hits = [], 0
                    while pending and len(ids_l) < self.lane_events:
                        h = sizes[pool_idx[pending[0]]]
                        if ids_l and hits + h > self.max_total_hits:
                            break
                        ids_l.append(pending.popleft())
                        hits += int(h)
                    ids = np.asarray(ids_l, dtype=np.int64)
                    m = len(ids)
                    batch_sizes.append(m)
                    max_batch_hits = max(max_batch_hits, hits)
                    self._launch(lane, ids, pool_idx[ids], pool, time.perf_counter() - t0)
                    progressed = True
            if not progressed and nxt < N and not pending and all(not l.busy for l in self.lanes):
                # idle until the next arrival
                wait = arrival_s[nxt] - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        lat = done_t - arrival_s
        span = float(np.nanmax(done_t) - arrival_s[0]) if N else 0.0
        return dict(
            events=N, offered_rate_hz=round(N / max(float(arrival_s[-1] - arrival_s[0]), 1e-9), 1) if N > 1 else None,
            events_per_s=round(N / span, 2) if span > 0 else None,
            hit_votes_per_s=round(votes / span, 1) if span > 0 else None,
            latency_ms_p50=round(float(np.percentile(lat, 50)) * 1e3, 4),
            latency_ms_p99=round(float(np.percentile(lat, 99)) * 1e3, 4),
            latency_ms_max=round(float(np.max(lat)) * 1e3, 4),
            mean_batch=round(float(np.mean(batch_sizes)), 2) if batch_sizes else 0.0,
            batches=len(batch_sizes), max_batch_hits=max_batch_hits, candidates=candidates, status_flags_or=flags_or,
            lanes=self.n_lanes, slots=self.slots, slot_bytes=self.slot_bytes,
            resident_bytes=self.slots * self.slot_bytes)


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int = 13054855) -> np.ndarray:
    rng = np.random.default_rng([seed, 5])
    n = int(rate_hz * duration_s * 1.1) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
    return t[t < duration_s]
