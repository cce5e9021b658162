"""Batched form (persistent work-queue vote over (event, slab), hipGraph replay,
launch-shape tuning): every event of a batch must come out bit-identical to the
single-event path and to the CPU oracle."""
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


def _single(H, plan, ev, thr, cap_peaks, cap_pairs):
    bufs = H.EventBuffers(plan, cap_peaks=cap_peaks, cap_pairs=cap_pairs)
    x, y, lay, _ = H.hits_to_device(ev)
    bufs.run(H.make_hits(x, y, lay), thr)
    torch.cuda.synchronize()
    r = bufs.results()
    r["acc"] = bufs.acc.cpu().numpy()
    return r


def _assert_same(a, b, ctx=""):
    for key in ("peaks", "offsets", "hit_idx"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=f"{ctx} {key}")
    for key in ("n_peaks", "n_pairs", "n_votes", "n_bad_hits", "flags"):
        assert a["status"][key] == b["status"][key], (ctx, key)


def _small_batch_events():
    cfg = configs.small_variant(configs.C3, n_phi=256, n_qpt=64, n_d0=8)
    sizes = [40, 0, 7, 120, 3, 65]
    events = []
    for i, nt in enumerate(sizes):
        events.append(synth.make_event(cfg.with_(n_tracks=nt, track_dist="fixed"), i))
    return cfg, events


def test_batch_equals_single_and_oracle(H, oracle_mod):
    O = oracle_mod
    cfg, events = _small_batch_events()
    plan = H.Plan(cfg, max_hits=4096)
    cap_peaks, cap_pairs = 1 << 14, 1 << 17
    bufs = H.BatchBuffers(plan, len(events), sum(e.n for e in events), cap_peaks, cap_pairs)
    bufs.load(events)
    print(f"[batch] small: {[e.n for e in events]} hits", flush=True)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    acc = bufs.acc.cpu().numpy()
    g = O.Cfg(cfg)
    for e, ev in enumerate(events):
        res = bufs.results(e)
        acc_ref, nv = O.vote(g, ev)
        np.testing.assert_array_equal(acc[e], acc_ref, err_msg=f"event {e}")
        n_ref, pk_ref = O.peaks(g, acc_ref, cfg.threshold)
        np.testing.assert_array_equal(res["peaks"], pk_ref)
        offs_ref, hit_ref, tot = O.assign(g, ev, pk_ref)
        np.testing.assert_array_equal(res["offsets"], offs_ref)
        np.testing.assert_array_equal(res["hit_idx"], hit_ref)
        assert res["status"]["n_votes"] == nv and res["status"]["n_hits"] == ev.n
        single = _single(H, plan, ev, cfg.threshold, cap_peaks, cap_pairs)
        _assert_same(res, single, f"event {e}")
        np.testing.assert_array_equal(acc[e], single["acc"])


def test_batch_wide_windows_read_the_16bit_counts(H, oracle_mod):
    """Batches vote from 8-bit window counts unless a window of the event holds more than 255 hits:
    an event with 300 extra hits at one azimuth of the innermost layer takes the 16-bit counts, its
    neighbours in the batch keep the 8-bit ones, and every event equals the oracle and the single
    path."""
    O = oracle_mod
    cfg, base = _small_batch_events()
    ev = base[3]
    phi = 0.7 + np.arange(300) * 1e-6
    r0 = cfg.radii_cm[0]
    x = np.concatenate([ev.x, (r0 * np.cos(phi)).astype(np.float32)])
    y = np.concatenate([ev.y, (r0 * np.sin(phi)).astype(np.float32)])
    lay = np.concatenate([ev.layer, np.zeros(300, np.uint8)])
    tid = np.concatenate([ev.track_id, np.full(300, -1, np.int32)])
    crowded = synth.Event(x=x, y=y, z=None, layer=lay, track_id=tid, truth=ev.truth)
    events = [base[0], crowded, base[5]]
    plan = H.Plan(cfg, max_hits=4096)
    cap_peaks, cap_pairs = 1 << 14, 1 << 18
    bufs = H.BatchBuffers(plan, len(events), sum(e.n for e in events), cap_peaks, cap_pairs)
    bufs.load(events)
    print(f"[batch] wide windows: {[e.n for e in events]} hits", flush=True)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    acc = bufs.acc.cpu().numpy()
    g = O.Cfg(cfg)
    for e, evt in enumerate(events):
        res = bufs.results(e)
        acc_ref, nv = O.vote(g, evt)
        np.testing.assert_array_equal(acc[e], acc_ref, err_msg=f"event {e}")
        n_ref, pk_ref = O.peaks(g, acc_ref, cfg.threshold)
        np.testing.assert_array_equal(res["peaks"], pk_ref)
        offs_ref, hit_ref, _ = O.assign(g, evt, pk_ref)
        np.testing.assert_array_equal(res["offsets"], offs_ref)
        np.testing.assert_array_equal(res["hit_idx"], hit_ref)
        single = _single(H, plan, evt, cfg.threshold, cap_peaks, cap_pairs)
        _assert_same(res, single, f"event {e}")
    assert acc[1].max() >= 300  # the crowded window really voted


def test_batch_event_too_large_is_flagged(H):
    cfg, events = _small_batch_events()
    plan = H.Plan(cfg, max_hits=200)
    big = [e for e in events if e.n > 200]
    assert big
    bufs = H.BatchBuffers(plan, len(events), sum(e.n for e in events), 1 << 12, 1 << 15)
    bufs.load(events)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    acc = bufs.acc.cpu().numpy()
    for e, ev in enumerate(events):
        st = bufs.results(e)["status"]
        if ev.n > 200:
            assert st["flags"] & H.HOUGH_F_EVENT_TOO_LARGE
            assert st["n_peaks"] == 0 and st["n_votes"] == 0 and not acc[e].any()
        else:
            assert not st["flags"] & H.HOUGH_F_EVENT_TOO_LARGE


def test_batch_full_grid_uneven_events(H, oracle_mod):
    """Sixteen events of the batched workload in the tuned launch shape (Gamma-Poisson track counts, full
    512x256x64 grid): accumulators, candidates and CSR offsets of every event
    equal the oracle; hit lists equal the single-event path (itself checked
    against the oracle) and the oracle on sampled candidates."""
    O = oracle_mod
    cfg = configs.C3
    events = [synth.make_event(cfg, i) for i in range(16)]
    plan = H.Plan(cfg, max_hits=32767)
    from paper_1305_4855_amd import tune
    shape = tune.apply(plan)  # the benchmark's launch shape
    cap_peaks, cap_pairs = 1 << 19, 1 << 23
    bufs = H.BatchBuffers(plan, len(events), sum(e.n for e in events), cap_peaks, cap_pairs)
    bufs.load(events)
    print(f"[batch] c3 x16 {shape}: {[e.n for e in events]} hits", flush=True)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    g = O.Cfg(cfg)
    rng = np.random.default_rng(31)
    for e in range(len(events)):
        res = bufs.results(e)
        acc = bufs.acc[e].cpu().numpy()
        acc_ref, nv = O.vote(g, events[e])
        assert int(np.count_nonzero(acc != acc_ref)) == 0, f"event {e}"
        n_ref, pk_ref = O.peaks(g, acc_ref, cfg.threshold)
        assert res["status"]["n_peaks"] == n_ref
        np.testing.assert_array_equal(res["peaks"], pk_ref)
        np.testing.assert_array_equal(np.diff(res["offsets"]), pk_ref[:, 3])
        if e % 4 == 0:
            single = _single(H, plan, events[e], cfg.threshold, cap_peaks, cap_pairs)
            _assert_same(res, single, f"event {e}")
        sel = np.unique(rng.choice(n_ref, min(n_ref, 100), replace=False))
        offs_s, hit_s, _ = O.assign(g, events[e], pk_ref[sel])
        offs = res["offsets"]
        for j, p in enumerate(sel):
            np.testing.assert_array_equal(res["hit_idx"][offs[p]:offs[p + 1]], hit_s[offs_s[j]:offs_s[j + 1]])


def test_graph_replays_match_eager(H):
    cfg, events = _small_batch_events()
    plan = H.Plan(cfg, max_hits=4096)
    cap_peaks, cap_pairs = 1 << 13, 1 << 16
    n_max = 2 * sum(e.n for e in events)
    bufs = H.BatchBuffers(plan, len(events), n_max, cap_peaks, cap_pairs)
    bufs.load(events)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    eager = [bufs.results(e) for e in range(len(events))]
    eager_acc = bufs.acc.cpu().numpy().copy()
    stream = torch.cuda.Stream()
    graph = H.Graph(bufs, cfg.threshold, stream)
    other = [synth.make_event(cfg.with_(n_tracks=nt, track_dist="fixed"), 100 + i)
             for i, nt in enumerate([5, 90, 0, 33, 60, 12])]
    other_ref = None
    for rep in range(4):
        # eager work of the program between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        evs = events if rep % 2 == 0 else other
        bufs.load(evs)
        bufs.status.fill_(-7)
        bufs.acc.fill_(-1)
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        got = [bufs.results(e) for e in range(len(evs))]
        if rep % 2 == 0:
            ref, ref_acc = eager, eager_acc
        else:
            if other_ref is None:
                bufs.run(cfg.threshold)
                torch.cuda.synchronize()
                other_ref = ([bufs.results(e) for e in range(len(evs))], bufs.acc.cpu().numpy().copy())
                got = other_ref[0]
            ref, ref_acc = other_ref
        for e in range(len(evs)):
            _assert_same(got[e], ref[e], f"replay {rep} event {e}")
        np.testing.assert_array_equal(bufs.acc.cpu().numpy(), ref_acc)
        del junk
    graph.close()


@pytest.mark.parametrize("tune", [dict(vote_threads=512, vote_grid=64, peak_planes=4),
                                  dict(vote_threads=256, vote_grid=7, peak_planes=16),
                                  dict(vote_threads=512, vote_grid=512, peak_planes=32),
                                  dict(vote_threads=1024, vote_grid=0, peak_planes=3),
                                  dict(vote_threads=512, vote_grid=100, peak_planes=8, vote_cols=4, assign_blocks=3,
                                       prep_rows=16),
                                  dict(vote_threads=1024, vote_grid=2048, peak_planes=32, vote_cols=64,
                                       assign_blocks=1, prep_rows=256)])
def test_results_identical_across_launch_shapes(H, tune):
    cfg, events = _small_batch_events()
    plan = H.Plan(cfg, max_hits=4096)
    bufs = H.BatchBuffers(plan, len(events), sum(e.n for e in events), 1 << 13, 1 << 16)
    bufs.load(events)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    ref = [bufs.results(e) for e in range(len(events))]
    ref_acc = bufs.acc.cpu().numpy().copy()
    plan.set_tuning(**tune)
    bufs.acc.fill_(-1)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    for e in range(len(events)):
        _assert_same(bufs.results(e), ref[e], f"{tune} event {e}")
    np.testing.assert_array_equal(bufs.acc.cpu().numpy(), ref_acc)
    # single-event path with the same tuning
    single = _single(H, plan, events[0], cfg.threshold, 1 << 13, 1 << 16)
    _assert_same(single, ref[0], f"{tune} single")
