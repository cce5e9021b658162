"""Trigger-style serving loop with continuous batching over resident slots.

Device memory holds two kinds of buffers, both allocated once:

* resident slots: one event's accumulator, candidate list, CSR offsets, CSR hit list and status
  (`slot_bytes`); as many slots as the memory budget holds after the launch contexts;
* launch contexts: one stream each, with what one batched chain in flight needs besides the slots
  (its workspace, the packed hits of its events, pinned host staging).

Arriving events wait in a host queue, oldest first.  Whenever a launch context is idle and events are
waiting, the oldest waiting events are admitted into it, as many as `max_batch`, the context's hit
buffer and the longest run of free slots allow (the batched chain writes the events of one launch
into consecutive slots).  Their hits are staged in pinned host memory and copied in on the context's
stream, the batched chain (`hough_run_batch`) writes each event's results into its slot, and the
statuses and first `topk` candidates come back to pinned host memory.  When a launch completes, its
slots are handed to `on_complete` and then freed, while other launches are still running: admission
is bounded by free slots (the memory budget) and idle contexts, never by another batch finishing.
Contexts run concurrently, so the copy-in of one launch overlaps the compute of another and the
copy-out of a third (the event pipelining of the paper's throughput figure, Sec. "Preliminary
Results").

Latency of an event = time from its arrival to the moment its candidate list and hit lists are
complete in its device slot and its status and first candidates are on the host.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np
import torch

from . import hough as H


def slot_bytes(plan: H.Plan, cap_peaks: int, cap_pairs: int) -> int:
    """Device bytes one resident event occupies: accumulator, candidates, CSR offsets and hit list, status."""
    return plan.acc_bytes + cap_peaks * 16 + (cap_peaks + 1) * 4 + cap_pairs * 4 + H.STATUS_BYTES


def context_bytes(plan: H.Plan, max_batch: int, cap_peaks: int, max_hits: int) -> int:
    """Device bytes of one launch context: the batch workspace and the packed hits (x, y, layer, offsets)."""
    return plan.batch_ws_bytes(max_batch, cap_peaks) + 9 * max_hits + 4 * (max_batch + 1)


@dataclasses.dataclass
class Context:
    idx: int
    stream: torch.cuda.Stream
    done: torch.cuda.Event
    ws: torch.Tensor
    x: torch.Tensor
    y: torch.Tensor
    layer: torch.Tensor
    hit_offsets: torch.Tensor
    x_h: torch.Tensor
    y_h: torch.Tensor
    lay_h: torch.Tensor
    off_h: torch.Tensor
    status_h: torch.Tensor
    top_h: torch.Tensor
    busy: bool = False
    ids: Optional[np.ndarray] = None
    slot0: int = 0
    t_launch: float = 0.0


class Slots:
    """Resident per-event outputs of `n` slots (consecutive slots form one launch's strided outputs)."""

    def __init__(self, plan: H.Plan, n: int, cap_peaks: int, cap_pairs: int, device="cuda"):
        c = plan.cfg
        self.n, self.cap_peaks, self.cap_pairs = int(n), int(cap_peaks), int(cap_pairs)
        self.acc = torch.empty((n, c.n_d0, c.n_qpt, c.n_phi), dtype=plan.acc_dtype, device=device)
        self.peaks = torch.empty((n, cap_peaks, H.PEAK_INTS), dtype=torch.int32, device=device)
        self.offsets = torch.empty((n, cap_peaks + 1), dtype=torch.int32, device=device)
        self.hit_idx = torch.empty((n, cap_pairs), dtype=torch.int32, device=device)
        self.status = torch.zeros((n, H.STATUS_BYTES // 4), dtype=torch.int32, device=device)
        self.free = np.ones(n, dtype=bool)

    def take(self, m: int) -> tuple:
        """First run of at least one free slot, as long as possible up to m: (start, length), or (-1, 0)."""
        f = self.free
        if not f.any():
            return -1, 0
        d = np.diff(np.concatenate(([0], f.view(np.int8), [0])))
        starts, ends = np.flatnonzero(d == 1), np.flatnonzero(d == -1)
        lens = ends - starts
        ok = np.flatnonzero(lens >= m)
        i = int(ok[0]) if ok.size else int(np.argmax(lens))
        s, n = int(starts[i]), int(min(m, lens[i]))
        f[s:s + n] = False
        return s, n

    def release(self, s: int, n: int) -> None:
        self.free[s:s + n] = True

    def results(self, s: int) -> dict:
        st = H.status_dict(self.status[s])
        n = min(st["n_peaks"], self.cap_peaks)
        npairs = min(st["n_pairs"], self.cap_pairs)
        return dict(status=st, peaks=self.peaks[s, :n].cpu().numpy(),
                    offsets=self.offsets[s, : n + 1].cpu().numpy().astype(np.int64),
                    hit_idx=self.hit_idx[s, :npairs].cpu().numpy())


class Server:
    """Continuous-batching server: `n_contexts` launch contexts of at most `max_batch` events each and
    as many resident slots as `budget_bytes` holds after the contexts (at most `max_slots`)."""

    def __init__(self, plan: H.Plan, threshold: int, budget_bytes: int, n_contexts: int = 4, max_batch: int = 64,
                 cap_peaks: int = 1 << 19, cap_pairs: int = 1 << 24, hits_per_event: int = 8192, topk: int = 64,
                 max_slots: Optional[int] = None):
        self.plan, self.threshold, self.topk = plan, int(threshold), int(topk)
        self.cap_peaks, self.cap_pairs = int(cap_peaks), int(cap_pairs)
        self.max_batch = int(max_batch)
        # packed hit buffer of a context: room for the largest event even when it is admitted alone
        self.max_ctx_hits = max(self.max_batch * int(hits_per_event), plan.max_hits)
        self.slot_bytes = slot_bytes(plan, cap_peaks, cap_pairs)
        self.context_bytes = context_bytes(plan, self.max_batch, cap_peaks, self.max_ctx_hits)
        n_slots = (int(budget_bytes) - int(n_contexts) * self.context_bytes) // self.slot_bytes
        if max_slots is not None:
            n_slots = min(n_slots, int(max_slots))
        if n_slots < 1:
            raise ValueError("memory budget below one launch context per stream plus one resident slot")
        self.budget_bytes = int(budget_bytes)
        self.slots = Slots(plan, int(n_slots), cap_peaks, cap_pairs)
        self.contexts: List[Context] = []
        nh = self.max_ctx_hits
        for i in range(int(n_contexts)):
            self.contexts.append(Context(
                idx=i, stream=torch.cuda.Stream(), done=torch.cuda.Event(),
                ws=torch.empty(plan.batch_ws_bytes(self.max_batch, cap_peaks), dtype=torch.uint8, device="cuda"),
                x=torch.zeros(nh, dtype=torch.float32, device="cuda"),
                y=torch.zeros(nh, dtype=torch.float32, device="cuda"),
                layer=torch.zeros(nh, dtype=torch.uint8, device="cuda"),
                hit_offsets=torch.zeros(self.max_batch + 1, dtype=torch.int32, device="cuda"),
                x_h=torch.empty(nh, dtype=torch.float32, pin_memory=True),
                y_h=torch.empty(nh, dtype=torch.float32, pin_memory=True),
                lay_h=torch.empty(nh, dtype=torch.uint8, pin_memory=True),
                off_h=torch.empty(self.max_batch + 1, dtype=torch.int32, pin_memory=True),
                status_h=torch.empty((self.max_batch, H.STATUS_BYTES // 4), dtype=torch.int32, pin_memory=True),
                top_h=torch.empty((self.max_batch, max(1, topk), H.PEAK_INTS), dtype=torch.int32,
                                  pin_memory=True)))

    @property
    def n_slots(self) -> int:
        return self.slots.n

    @property
    def resident_bytes(self) -> int:
        return self.slots.n * self.slot_bytes + len(self.contexts) * self.context_bytes

    # ------------------------------------------------------------------ one launch
    def _launch(self, ctx: Context, ids: np.ndarray, s0: int, pool_ids: np.ndarray, pool, now: float) -> None:
        evs = [pool[i] for i in pool_ids]
        m = len(evs)
        offs = np.zeros(m + 1, dtype=np.int32)
        np.cumsum(np.fromiter((e.n for e in evs), dtype=np.int64, count=m), out=offs[1:])
        n = int(offs[-1])
        if n > self.max_ctx_hits:
            raise RuntimeError("admitted events exceed the context's hit buffer")
        if n:
            ctx.x_h.numpy()[:n] = np.concatenate([e.x for e in evs])
            ctx.y_h.numpy()[:n] = np.concatenate([e.y for e in evs])
            ctx.lay_h.numpy()[:n] = np.concatenate([e.layer for e in evs])
        ctx.off_h.numpy()[: m + 1] = offs
        S = self.slots
        sl = slice(s0, s0 + m)
        with torch.cuda.stream(ctx.stream):
            if n:
                ctx.x[:n].copy_(ctx.x_h[:n], non_blocking=True)
                ctx.y[:n].copy_(ctx.y_h[:n], non_blocking=True)
                ctx.layer[:n].copy_(ctx.lay_h[:n], non_blocking=True)
            ctx.hit_offsets[: m + 1].copy_(ctx.off_h[: m + 1], non_blocking=True)
            b = H.Batch(H._ptr(ctx.x), H._ptr(ctx.y), None, H._ptr(ctx.layer), H._ptr(ctx.hit_offsets), m,
                        self.threshold, self.cap_peaks, self.cap_pairs, H._ptr(S.acc[sl]), H._ptr(S.peaks[sl]),
                        H._ptr(S.offsets[sl]), H._ptr(S.hit_idx[sl]), H._ptr(ctx.ws), ctx.ws.numel(),
                        H._ptr(S.status[sl]), None)
            H.run_batch(self.plan, b, ctx.stream)
            ctx.status_h[:m].copy_(S.status[sl], non_blocking=True)
            if self.topk:
                ctx.top_h[:m].copy_(S.peaks[sl, : self.topk], non_blocking=True)
            ctx.done.record(ctx.stream)
        ctx.busy, ctx.ids, ctx.slot0, ctx.t_launch = True, ids, s0, now

    # ------------------------------------------------------------------ the loop
    def serve(self, pool, arrival_s: np.ndarray, pool_idx: np.ndarray,
              on_complete: Optional[Callable[["Server", Context, np.ndarray, np.ndarray], None]] = None,
              progress: Optional[Callable[[float, int, int], None]] = None, progress_every_s: float = 10.0) -> Dict:
        """Serve events arriving at `arrival_s` (seconds from the start, increasing), each a copy of
        `pool[pool_idx[i]]`, paced in wall-clock time.  `on_complete(server, ctx, ids, pool_ids)` runs
        when a launch is done, while its events' results are still in slots ctx.slot0 + j;
        `progress(t, served, queued)` runs every `progress_every_s` seconds.  Returns latency and
        throughput figures."""
        N = len(arrival_s)
        sizes = np.fromiter((e.n for e in pool), dtype=np.int64, count=len(pool))
        done_t = np.full(N, np.nan)
        flags_or, flagged, votes, candidates = 0, 0, 0, 0
        pending: collections.deque = collections.deque()
        nxt, served = 0, 0
        batch_sizes: List[int] = []
        max_batch_hits, max_slots_used, slots_short = 0, 0, 0
        S = self.slots
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
            for ctx in self.contexts:
                if ctx.busy and ctx.done.query():
                    tdone = time.perf_counter() - t0
                    m = len(ctx.ids)
                    st = ctx.status_h[:m].numpy()
                    done_t[ctx.ids] = tdone
                    votes += int(st.view(np.int64)[:, 1].sum())
                    candidates += int(st[:, 4].sum())
                    fl = st[:, 5]
                    flags_or |= int(np.bitwise_or.reduce(fl)) if m else 0
                    flagged += int(np.count_nonzero(fl))
                    if on_complete is not None:
                        on_complete(self, ctx, ctx.ids, pool_idx[ctx.ids])
                    S.release(ctx.slot0, m)
                    served += m
                    ctx.busy = False
                    progressed = True
            for ctx in self.contexts:
                if ctx.busy or not pending:
                    continue
                # oldest first, as many as max_batch and the context's hit buffer hold
                want, hits = 0, 0
                for q in range(min(len(pending), self.max_batch)):
                    h = int(sizes[pool_idx[pending[q]]])
                    if want and hits + h > self.max_ctx_hits:
                        break
                    want += 1
                    hits += h
                s0, m = S.take(want)
                if m == 0:
                    slots_short += 1
                    break  # no free slot: wait for a launch to complete
                ids = np.fromiter((pending.popleft() for _ in range(m)), dtype=np.int64, count=m)
                batch_sizes.append(m)
                max_batch_hits = max(max_batch_hits, int(sizes[pool_idx[ids]].sum()))
                max_slots_used = max(max_slots_used, int(S.n - S.free.sum()))
                self._launch(ctx, ids, s0, pool_idx[ids], pool, time.perf_counter() - t0)
                progressed = True
            if not progressed and nxt < N and not pending and all(not c.busy for c in self.contexts):
                wait = arrival_s[nxt] - (time.perf_counter() - t0)  # idle until the next arrival
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
            batches=len(batch_sizes), max_batch_hits=max_batch_hits, candidates=candidates,
            status_flags_or=flags_or, events_flagged=flagged, contexts=len(self.contexts), max_batch=self.max_batch,
            slots=S.n, max_slots_in_use=max_slots_used, admissions_short_of_slots=slots_short,
            slot_bytes=self.slot_bytes, context_bytes=self.context_bytes, resident_bytes=self.resident_bytes,
            budget_bytes=self.budget_bytes)


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int = 13054855) -> np.ndarray:
    rng = np.random.default_rng([seed, 5])
    n = int(rate_hz * duration_s * 1.1) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
    return t[t < duration_s]
