"""Serving loop (continuous batching): every event served in the mix of a
stream must give exactly the result it gives alone."""
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


def test_server_rejects_budget_below_one_accumulator(H):
    from paper_1305_4855_amd import serve

    cfg = configs.small_variant(configs.C5, n_phi=256, n_qpt=64, n_d0=8)
    plan = H.Plan(cfg, max_hits=4096)
    with pytest.raises(ValueError):
        serve.Server(plan, cfg.threshold, acc_budget_bytes=plan.acc_bytes - 1)


def test_served_results_equal_alone(H):
    from paper_1305_4855_amd import serve

    cfg = configs.small_variant(configs.C5, n_phi=256, n_qpt=64, n_d0=8)
    pool = [synth.make_event(cfg.with_(n_tracks=nt, track_dist="fixed"), i)
            for i, nt in enumerate([3, 40, 0, 120, 17, 75, 9, 200, 55, 31, 1, 88])]
    plan = H.Plan(cfg, max_hits=4096)
    cap_peaks, cap_pairs = 1 << 13, 1 << 16
    # each pool event alone, through the single-event path
    alone = []
    for ev in pool:
        bufs = H.EventBuffers(plan, cap_peaks=cap_peaks, cap_pairs=cap_pairs)
        x, y, lay, _ = H.hits_to_device(ev)
        bufs.run(H.make_hits(x, y, lay), cfg.threshold)
        torch.cuda.synchronize()
        alone.append(bufs.results())
    # accumulator budget of 15 events -> 3 lanes of 5 slots
    srv = serve.Server(plan, cfg.threshold, acc_budget_bytes=15 * plan.acc_bytes + 100, max_lanes=3,
                       cap_peaks=cap_peaks, cap_pairs=cap_pairs, hits_per_slot=600, topk=16)
    assert srv.n_lanes == 3 and srv.lane_events == 5 and srv.slots == 15
    assert srv.max_total_hits == 4096
    rng = np.random.default_rng(41)
    n = 240
    arrivals = np.sort(rng.uniform(0.0, 0.05, size=n))
    pool_idx = rng.integers(0, len(pool), size=n)
    checked = []

    def on_complete(lane, ids, pids):
        b = lane.bufs
        for j, pid in enumerate(pids):
            ref = alone[pid]
            st = H.status_dict(b.status[j])
            for key in ("n_peaks", "n_pairs", "n_votes", "n_bad_hits", "flags"):
                assert st[key] == ref["status"][key], (key, pid)
            npk = min(st["n_peaks"], cap_peaks)
            np.testing.assert_array_equal(b.peaks[j, :npk].cpu().numpy(), ref["peaks"])
            np.testing.assert_array_equal(b.offsets[j, : npk + 1].cpu().numpy(), ref["offsets"])
            np.testing.assert_array_equal(b.hit_idx[j, : min(st["n_pairs"], cap_pairs)].cpu().numpy(),
                                          ref["hit_idx"])
            top = lane.status_h  # the status copied back with the batch is the same
            np.testing.assert_array_equal(top[j].numpy(), b.status[j].cpu().numpy())
            k = min(16, npk)
            np.testing.assert_array_equal(lane.top_h[j, :k].numpy(), ref["peaks"][:k])
            checked.append(int(ids[j]))

    print(f"[serve] pool hits {[e.n for e in pool]}", flush=True)
    stats = srv.serve(pool, arrivals, pool_idx, on_complete=on_complete)
    print(f"[serve] {stats}", flush=True)
    assert sorted(checked) == list(range(n))
    assert stats["events"] == n and stats["batches"] >= n // 5
    # the hit buffer (4096 hits) bounds admission below the slot count for the large events
    assert stats["max_batch_hits"] <= 4096
    assert stats["latency_ms_p99"] >= stats["latency_ms_p50"] > 0
    # mixed batches really happened (more than one event per launch on average)
    assert stats["mean_batch"] > 1.0
