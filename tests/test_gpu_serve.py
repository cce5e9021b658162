"""Serving loop (continuous batching over resident slots): every event served in the mix of a stream
gives exactly the result it gives alone and the oracle's result (all outputs are integers: tolerance
zero)."""
import numpy as np
import pytest

from paper_1305_4855_amd import configs, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_4855_amd import hough as H
    return H


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.build()
    return O


def _oracle_event(O, cfg, ev, cap_peaks, sample=None, seed=0):
    """The oracle's accumulator, candidates and (all, or `sample` random) hit lists of one event."""
    g = O.Cfg(cfg)
    acc, nv = O.vote(g, ev)
    n, pk = O.peaks(g, acc, cfg.threshold)
    assert n <= cap_peaks
    if sample is None or sample >= n:
        sel = np.arange(n)
    else:
        sel = np.sort(np.random.default_rng(seed).choice(n, size=sample, replace=False))
    offs, hit_idx, tot = O.assign(g, ev, pk[sel])
    return dict(acc=acc, n_votes=nv, peaks=pk, sel=sel, offs=offs, hit_idx=hit_idx)


def _check_slot_against_oracle(srv, s, ref):
    S = srv.slots
    st = S.results(s)["status"]
    assert st["flags"] == 0
    assert st["n_votes"] == ref["n_votes"]
    np.testing.assert_array_equal(S.acc[s].cpu().numpy(), ref["acc"])
    n = st["n_peaks"]
    assert n == ref["peaks"].shape[0]
    np.testing.assert_array_equal(S.peaks[s, :n].cpu().numpy(), ref["peaks"])
    offs = S.offsets[s, : n + 1].cpu().numpy().astype(np.int64)
    hit_idx = S.hit_idx[s, : st["n_pairs"]].cpu().numpy()
    for j, i in enumerate(ref["sel"]):
        np.testing.assert_array_equal(hit_idx[offs[i]:offs[i + 1]], ref["hit_idx"][ref["offs"][j]:ref["offs"][j + 1]])


def test_server_rejects_budget_below_one_slot(H):
    from paper_1305_4855_amd import serve

    cfg = configs.small_variant(configs.C5, n_phi=256, n_qpt=64, n_d0=8)
    plan = H.Plan(cfg, max_hits=4096)
    need = serve.slot_bytes(plan, 1 << 10, 1 << 12) + 2 * serve.context_bytes(plan, 4, 1 << 10, 4096)
    with pytest.raises(ValueError):
        serve.Server(plan, cfg.threshold, budget_bytes=need - 1, n_contexts=2, max_batch=4, cap_peaks=1 << 10,
                     cap_pairs=1 << 12, hits_per_event=1024)
    srv = serve.Server(plan, cfg.threshold, budget_bytes=need, n_contexts=2, max_batch=4, cap_peaks=1 << 10,
                       cap_pairs=1 << 12, hits_per_event=1024)
    assert srv.n_slots == 1 and srv.resident_bytes <= need


def test_served_results_equal_alone_and_oracle(H, O):
    from paper_1305_4855_amd import serve

    cfg = configs.small_variant(configs.C5, n_phi=256, n_qpt=64, n_d0=8)
    pool = [synth.make_event(cfg.with_(n_tracks=nt, track_dist="fixed"), i)
            for i, nt in enumerate([3, 40, 0, 120, 17, 75, 9, 200, 55, 31, 1, 88])]
    plan = H.Plan(cfg, max_hits=4096)
    cap_peaks, cap_pairs = 1 << 13, 1 << 16
    # each pool event alone, through the single-event path, and through the oracle
    alone = []
    for ev in pool:
        bufs = H.EventBuffers(plan, cap_peaks=cap_peaks, cap_pairs=cap_pairs)
        x, y, lay, _ = H.hits_to_device(ev)
        bufs.run(H.make_hits(x, y, lay), cfg.threshold)
        torch.cuda.synchronize()
        alone.append(bufs.results())
    ref = [_oracle_event(O, cfg, ev, cap_peaks) for ev in pool]
    # 3 contexts of at most 5 events, 15 slots: admission is bounded by free slots
    budget = 15 * serve.slot_bytes(plan, cap_peaks, cap_pairs) + 3 * serve.context_bytes(plan, 5, cap_peaks, 4096)
    srv = serve.Server(plan, cfg.threshold, budget_bytes=budget, n_contexts=3, max_batch=5, cap_peaks=cap_peaks,
                       cap_pairs=cap_pairs, hits_per_event=600, topk=16)
    assert srv.n_slots == 15 and srv.max_ctx_hits == 4096
    rng = np.random.default_rng(41)
    n = 240
    arrivals = np.sort(rng.uniform(0.0, 0.05, size=n))
    pool_idx = rng.integers(0, len(pool), size=n)
    checked = []

    def on_complete(server, ctx, ids, pids):
        S = server.slots
        for j, pid in enumerate(pids):
            s = ctx.slot0 + j
            got = S.results(s)
            r = alone[pid]
            for key in ("n_peaks", "n_pairs", "n_votes", "n_bad_hits", "flags"):
                assert got["status"][key] == r["status"][key], (key, pid)
            np.testing.assert_array_equal(got["peaks"], r["peaks"])
            np.testing.assert_array_equal(got["offsets"], r["offsets"])
            np.testing.assert_array_equal(got["hit_idx"], r["hit_idx"])
            _check_slot_against_oracle(server, s, ref[pid])
            # the status and first candidates copied back with the launch are the resident ones
            np.testing.assert_array_equal(ctx.status_h[j].numpy(), S.status[s].cpu().numpy())
            k = min(16, got["status"]["n_peaks"])
            np.testing.assert_array_equal(ctx.top_h[j, :k].numpy(), r["peaks"][:k])
            checked.append(int(ids[j]))

    print(f"[serve] pool hits {[e.n for e in pool]}", flush=True)
    stats = srv.serve(pool, arrivals, pool_idx, on_complete=on_complete)
    print(f"[serve] {stats}", flush=True)
    assert sorted(checked) == list(range(n))
    assert stats["events"] == n and stats["events_flagged"] == 0 and stats["status_flags_or"] == 0
    assert stats["max_batch_hits"] <= 4096 and stats["max_slots_in_use"] <= 15
    assert stats["latency_ms_p99"] >= stats["latency_ms_p50"] > 0
    assert stats["mean_batch"] > 1.0  # mixed launches really happened


def test_served_full_grid_largest_events_equal_oracle(H, O):
    """The streaming workload's own grid (512 x 256 x 64 int32) with a pool that includes the largest
    size class of the batched workload (2000 tracks, about 24k hits, 13M hit-candidate pairs): every
    served event's accumulator, vote total and candidate list equal the oracle's in full, and 200
    sampled hit lists per event; no event is cut."""
    from paper_1305_4855_amd import serve

    cfg = configs.C5
    sizes = [2000, 50, 480, 1200, 0, 2000]
    pool = [synth.make_event(cfg.with_(n_tracks=nt, track_dist="fixed"), 900 + i) for i, nt in enumerate(sizes)]
    print(f"[serve-full] pool hits {[e.n for e in pool]}", flush=True)
    plan = H.Plan(cfg, max_hits=cfg.max_hits_per_event)
    cap_peaks, cap_pairs = 1 << 19, 1 << 24
    ref = [_oracle_event(O, cfg, ev, cap_peaks, sample=200, seed=i) for i, ev in enumerate(pool)]
    budget = (6 * serve.slot_bytes(plan, cap_peaks, cap_pairs) +
              2 * serve.context_bytes(plan, 3, cap_peaks, max(3 * 8192, plan.max_hits)))
    srv = serve.Server(plan, cfg.threshold, budget_bytes=budget, n_contexts=2, max_batch=3, cap_peaks=cap_peaks,
                       cap_pairs=cap_pairs, hits_per_event=8192, topk=8)
    assert srv.n_slots == 6
    arrivals = np.linspace(0.0, 0.02, 14)
    pool_idx = np.array([0, 1, 2, 3, 4, 5, 5, 0, 3, 1, 2, 4, 0, 5])
    checked = []

    def on_complete(server, ctx, ids, pids):
        for j, pid in enumerate(pids):
            _check_slot_against_oracle(server, ctx.slot0 + j, ref[pid])
            checked.append(int(ids[j]))

    stats = srv.serve(pool, arrivals, pool_idx, on_complete=on_complete)
    print(f"[serve-full] {stats}", flush=True)
    assert sorted(checked) == list(range(len(arrivals)))
    assert stats["events_flagged"] == 0 and stats["status_flags_or"] == 0
