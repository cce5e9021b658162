"""Track fit (algebraic circle fit of each candidate's hit list): GPU against the CPU oracle,
bit for bit (both sum the moments in list order in IEEE double without contraction), through
the C ABI (hough_fit)."""
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


def _chain_with_fit(H, cfg, ev, cap_peaks, cap_pairs, max_hits=None):
    plan = H.Plan(cfg, max_hits=max_hits or max(ev.n, 1))
    bufs = H.EventBuffers(plan, cap_peaks=cap_peaks, cap_pairs=cap_pairs)
    x, y, lay, _ = H.hits_to_device(ev)
    hits = H.make_hits(x, y, lay)
    bufs.run(hits, cfg.threshold)
    bufs.run_fit(hits)
    torch.cuda.synchronize()
    return bufs.results()


@pytest.mark.parametrize("shape,tracks,eid", [((256, 64, 4), 30, 0), ((512, 64, 8), 60, 1), ((16, 64, 2), 5, 2)])
def test_fit_small_events_equal_oracle(H, oracle_mod, shape, tracks, eid):
    O = oracle_mod
    cfg = configs.small_variant(configs.C2, n_tracks=tracks, n_phi=shape[0], n_qpt=shape[1], n_d0=shape[2])
    ev = synth.make_event(cfg, eid)
    res = _chain_with_fit(H, cfg, ev, 1 << 16, 1 << 20)
    assert res["status"]["n_peaks"] > 0
    g = O.Cfg(cfg)
    _, pk = O.peaks(g, O.vote(g, ev)[0], cfg.threshold)
    offs, hit_idx, _ = O.assign(g, ev, pk)  # the oracle's own lists, equal to the GPU's
    np.testing.assert_array_equal(res["offsets"], offs)
    np.testing.assert_array_equal(res["hit_idx"], hit_idx)
    ref = O.fit(ev, offs, hit_idx)
    np.testing.assert_array_equal(res["fit"], ref)
    assert (ref[:, 2] > 0).any()


def test_fit_full_dense_event(H, oracle_mod):
    """Every candidate of the dense event (about 237k candidates, 7.0M hit-candidate pairs)."""
    O = oracle_mod
    cfg = configs.C2
    ev = synth.make_event(cfg, 0)
    print(f"[fit] c2 full n_hits={ev.n}", flush=True)
    res = _chain_with_fit(H, cfg, ev, 1 << 19, 1 << 24, max_hits=16384)
    g = O.Cfg(cfg)
    n, pk = O.peaks(g, O.vote(g, ev)[0], cfg.threshold)
    np.testing.assert_array_equal(res["peaks"], pk)
    offs, hit_idx, _ = O.assign(g, ev, pk)
    np.testing.assert_array_equal(res["fit"], O.fit(ev, offs, hit_idx))


def test_fit_cut_lists_marked(H, oracle_mod):
    O = oracle_mod
    cfg = configs.small_variant(configs.C2, n_tracks=40, n_phi=256, n_qpt=64, n_d0=4)
    ev = synth.make_event(cfg, 3)
    full = _chain_with_fit(H, cfg, ev, 1 << 16, 1 << 20)
    tot = int(full["offsets"][-1])
    cut = _chain_with_fit(H, cfg, ev, 1 << 16, tot // 2)
    offs = cut["offsets"]
    complete = offs[1:] <= tot // 2
    assert complete.any() and not complete.all()
    np.testing.assert_array_equal(cut["fit"][complete], full["fit"][complete])
    assert (cut["fit"][~complete, 2] == -2.0).all()
    np.testing.assert_array_equal(cut["fit"][~complete, 3], np.diff(offs)[~complete].astype(np.float64))


@pytest.mark.parametrize("n_hits", [400, 20000])
def test_fit_hand_made_lists(H, oracle_mod, n_hits):
    """Lists given directly to hough_fit: empty, two hits, collinear hits, integer points on a
    circle, and ordinary ones; the number of candidates comes from the status on the device.
    400 hits: the coordinates are copied into LDS; 20000 hits: more than fit there, so they are
    gathered from memory."""
    O = oracle_mod
    rng = np.random.default_rng(9)
    x = rng.uniform(-80, 80, n_hits).astype(np.float32)
    y = rng.uniform(-80, 80, n_hits).astype(np.float32)
    x[:5] = [13, 14, 15, 10, 7]  # on the circle of centre (10, -7), radius 5
    y[:5] = [-3, -4, -7, -2, -3]
    x[5:9] = [0, 1, 2, 4]  # collinear
    y[5:9] = [0, 1, 2, 4]
    lists = [[], [20, 21], [5, 6, 7, 8], [0, 1, 2, 3, 4]] + [list(rng.integers(0, n_hits, int(k)))
                                                            for k in rng.integers(3, 60, 300)]
    offs = np.concatenate([[0], np.cumsum([len(l) for l in lists])]).astype(np.int64)
    idx = np.concatenate([np.asarray(l, dtype=np.int32) for l in lists]).astype(np.int32)
    ev = synth.Event(x=x, y=y, z=None, layer=np.zeros(n_hits, np.uint8), track_id=np.full(n_hits, -1, np.int32),
                     truth={})
    ref = O.fit(ev, offs, idx)
    cfg = configs.small_variant(configs.C2, n_phi=256, n_qpt=64, n_d0=2)
    plan = H.Plan(cfg, max_hits=n_hits)
    cap_peaks = len(lists) + 7
    d_offs = torch.zeros(cap_peaks + 1, dtype=torch.int32, device="cuda")
    d_offs[: offs.size] = torch.from_numpy(offs.astype(np.int32)).cuda()
    d_idx = torch.from_numpy(idx).cuda()
    status = torch.zeros(H.STATUS_BYTES // 4, dtype=torch.int32, device="cuda")
    status[4] = len(lists)  # n_peaks (int32 at byte 16)
    out = torch.full((cap_peaks, 4), 7.0, dtype=torch.float64, device="cuda")
    xd, yd, ld, _ = H.hits_to_device(ev)
    H.fit(plan, H.make_hits(xd, yd, ld), d_offs, d_idx, status, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    np.testing.assert_array_equal(got[: len(lists)], ref)
    assert tuple(got[3]) == (10.0, -7.0, 25.0, 5.0)
    assert tuple(got[0]) == (0.0, 0.0, -1.0, 0.0) and got[1][2] == -1.0 and got[2][2] == -1.0
    assert (got[len(lists):] == 7.0).all()  # rows past the listed candidates are not written


@pytest.mark.parametrize("max_hits", [4096, 32767])
def test_fit_batch_equals_oracle(H, oracle_mod, max_hits):
    """hough_fit_batch after the batched chain: uneven events (one without hits, one cut by the
    pair capacity), each event's rows equal the oracle's fit of its own lists.  A plan of at most
    16384 hits per event stages each event's coordinates in LDS (k_fit_res, per-event hit base);
    one of 32767 gathers them from memory (k_fit)."""
    O = oracle_mod
    cfg = configs.small_variant(configs.C2, n_phi=256, n_qpt=64, n_d0=4)
    events = [synth.make_event(cfg.with_(n_tracks=t), i) for i, t in enumerate((30, 0, 55, 12))]
    plan = H.Plan(cfg, max_hits=max_hits)
    cap_pairs = 3000  # the 55-track event has about 6600 pairs: its later lists are cut
    bufs = H.BatchBuffers(plan, len(events), max(sum(e.n for e in events), 1), cap_peaks=1 << 12, cap_pairs=cap_pairs)
    bufs.load(events)
    bufs.run(cfg.threshold, zvote=False)
    bufs.run_fit()
    torch.cuda.synchronize()
    g = O.Cfg(cfg)
    cut_seen = False
    for e, ev in enumerate(events):
        r = bufs.results(e)
        _, pk = O.peaks(g, O.vote(g, ev)[0], cfg.threshold)
        offs, hit_idx, tot = O.assign(g, ev, pk)
        np.testing.assert_array_equal(r["peaks"], pk)
        ref = O.fit(ev, offs, hit_idx)
        cut = offs[1:] > cap_pairs
        cut_seen = cut_seen or bool(cut.any())
        np.testing.assert_array_equal(r["fit"][~cut], ref[~cut])
        assert (r["fit"][cut, 2] == -2.0).all()
    assert cut_seen
