"""Second-stage r-z vote (cot theta x z0 per candidate): GPU against the CPU
oracle, bit-exact, through the C ABI (hough_zvote, hough_run_batch)."""
import dataclasses

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


def _small_cfg():
    # the r-z grid of the large-grid workload (128 x 128, cot [-2, 2], z0 [-32, 32] cm) on a reduced
    # transverse grid
    return configs.small_variant(configs.C4, n_tracks=60, n_phi=256, n_qpt=64, n_d0=8)


def _run_single(H, plan, ev, thr, cap_peaks, cap_pairs):
    bufs = H.EventBuffers(plan, cap_peaks=cap_peaks, cap_pairs=cap_pairs)
    x, y, lay, z = H.hits_to_device(ev)
    bufs.run(H.make_hits(x, y, lay, z), thr)
    torch.cuda.synchronize()
    return bufs.results()


def test_arclen_table_matches_oracle(H, oracle_mod):
    O = oracle_mod
    cfg = _small_cfg()
    plan = H.Plan(cfg, max_hits=4096)
    S = plan.arclen_table()
    E = plan.table()
    g = O.Cfg(cfg)
    for L, r in enumerate(cfg.radii_cm):
        for l in range(cfg.n_d0):
            d = O.d0_centre(g, l)
            for k in range(cfg.n_qpt):
                ok, ref = O.arclen(r, O.curvature(g, k), d)
                assert (S[L, l, k] >= 0) == ok == (E[L, l, k] != np.iinfo(np.int32).min), (L, l, k)
                if ok:
                    assert S[L, l, k] == ref, (L, l, k)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_zvote_small_events_equal_oracle(H, oracle_mod, seed):
    O = oracle_mod
    cfg = _small_cfg()
    ev = synth.make_event(cfg, seed)
    print(f"[zvote] small event {seed}: {ev.n} hits", flush=True)
    plan = H.Plan(cfg, max_hits=4096)
    res = _run_single(H, plan, ev, cfg.threshold, 1 << 16, 1 << 20)
    g = O.Cfg(cfg)
    acc, _ = O.vote(g, ev)
    n, pk = O.peaks(g, acc, cfg.threshold)
    np.testing.assert_array_equal(res["peaks"], pk)
    offs, hit_idx, _ = O.assign(g, ev, pk)
    ref = O.zvote(g, ev, pk, offs, hit_idx)
    np.testing.assert_array_equal(res["zvote"], ref)
    assert (ref[:, 2] > 0).any() and n > 0


def test_zvote_bad_z_and_big_candidates(H, oracle_mod):
    """Unusable z values are skipped; candidates with more than 64 hits (nine
    copies of one track) take the row-by-row path."""
    O = oracle_mod
    cfg = _small_cfg()
    base = synth.make_event(cfg.with_(n_tracks=1, track_dist="fixed", noise_frac=0.0), 7)
    reps = 9
    x = np.concatenate([base.x] * reps)
    y = np.concatenate([base.y] * reps)
    z = np.concatenate([base.z + 0.01 * i for i in range(reps)]).astype(np.float32)
    lay = np.concatenate([base.layer] * reps)
    noise = synth.make_event(cfg.with_(n_tracks=30, track_dist="fixed"), 8)
    x, y, z, lay = (np.concatenate([a, b]) for a, b in ((x, noise.x), (y, noise.y), (z, noise.z),
                                                       (lay, noise.layer)))
    z = z.astype(np.float32)
    z[3] = np.nan
    z[17] = np.inf
    z[40] = 40000.0
    ev = dataclasses.replace(noise, x=x.astype(np.float32), y=y.astype(np.float32), z=z, layer=lay.astype(np.uint8))
    plan = H.Plan(cfg, max_hits=4096)
    res = _run_single(H, plan, ev, cfg.threshold, 1 << 16, 1 << 20)
    g = O.Cfg(cfg)
    acc, _ = O.vote(g, ev)
    n, pk = O.peaks(g, acc, cfg.threshold)
    np.testing.assert_array_equal(res["peaks"], pk)
    assert pk[:, 3].max() > 64
    offs, hit_idx, _ = O.assign(g, ev, pk)
    ref = O.zvote(g, ev, pk, offs, hit_idx)
    np.testing.assert_array_equal(res["zvote"], ref)


def test_zvote_cut_lists_marked(H, oracle_mod):
    O = oracle_mod
    cfg = _small_cfg()
    ev = synth.make_event(cfg, 3)
    plan = H.Plan(cfg, max_hits=4096)
    g = O.Cfg(cfg)
    acc, _ = O.vote(g, ev)
    n, pk = O.peaks(g, acc, cfg.threshold)
    offs, hit_idx, tot = O.assign(g, ev, pk)
    cap_pairs = int(tot // 3)
    res = _run_single(H, plan, ev, cfg.threshold, 1 << 16, cap_pairs)
    assert res["status"]["flags"] & H.HOUGH_F_PAIR_OVERFLOW
    ref = O.zvote(g, ev, pk, offs, hit_idx)
    complete = offs[1:] <= cap_pairs
    assert complete.any() and not complete.all()
    np.testing.assert_array_equal(res["zvote"][complete], ref[complete])
    assert (res["zvote"][~complete] == -1).all()


def test_zvote_batch_equals_single(H):
    cfg = _small_cfg()
    events = [synth.make_event(cfg.with_(n_tracks=nt, track_dist="fixed"), 20 + i)
              for i, nt in enumerate([30, 0, 5, 80])]
    plan = H.Plan(cfg, max_hits=4096)
    cap_peaks, cap_pairs = 1 << 15, 1 << 19
    bufs = H.BatchBuffers(plan, len(events), sum(e.n for e in events), cap_peaks, cap_pairs)
    bufs.load(events)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    for e, ev in enumerate(events):
        got = bufs.results(e)
        ref = _run_single(H, plan, ev, cfg.threshold, cap_peaks, cap_pairs)
        np.testing.assert_array_equal(got["peaks"], ref["peaks"])
        np.testing.assert_array_equal(got["zvote"], ref["zvote"])


def test_zvote_full_event_sampled(H, oracle_mod):
    """One event of the large-grid workload (1024 x 512 x 128, int16, 600
    tracks): zvote of sampled candidates equals the oracle's, computed from the
    oracle's own candidate list and hit lists."""
    O = oracle_mod
    cfg = configs.C4
    ev = synth.make_event(cfg, 0)
    print(f"[zvote] full c4 event: {ev.n} hits", flush=True)
    plan = H.Plan(cfg, max_hits=cfg.max_hits_per_event)
    res = _run_single(H, plan, ev, cfg.threshold, 1 << 21, 1 << 25)
    g = O.Cfg(cfg)
    acc, _ = O.vote(g, ev)
    n, pk = O.peaks(g, acc, cfg.threshold)
    assert res["status"]["n_peaks"] == n
    np.testing.assert_array_equal(res["peaks"], pk)
    rng = np.random.default_rng(5)
    sel = np.unique(rng.choice(n, 4000, replace=False))
    offs, hit_idx, _ = O.assign(g, ev, pk[sel])
    ref = O.zvote(g, ev, pk[sel], offs, hit_idx)
    np.testing.assert_array_equal(res["zvote"][sel], ref)


@pytest.mark.parametrize("change", [dict(z0_max=28.0),              # bin width 60/128 cm: not a power of two
                                    dict(cot_max=2.1),              # cot centres off the Q16.16 lattice
                                    dict(n_z0=1024, n_cot=32),      # too many z0 bins for the LDS rows
                                    dict(n_cot=1024)])              # n_cot * n_z0 > 65536
def test_unsupported_zgrids_rejected(H, change):
    cfg = dataclasses.replace(_small_cfg(), **change)
    with pytest.raises(H.HoughError, match="unsupported"):
        H.Plan(cfg, max_hits=4096)


def test_zvote_needs_small_events(H):
    cfg = dataclasses.replace(_small_cfg(), acc_bits=32, frac_bits=8)
    with pytest.raises(H.HoughError, match="unsupported"):
        H.Plan(cfg, max_hits=70000)


def test_zvote_in_captured_graph(H):
    """The batched chain with the r-z stage, captured once in a hipGraph and replayed with eager
    work and reloads in between, equals the eager chain every time."""
    cfg = _small_cfg()
    sets = [[synth.make_event(cfg.with_(n_tracks=nt, track_dist="fixed"), 60 + 10 * r + i)
             for i, nt in enumerate([25, 4, 70])] for r in range(2)]
    plan = H.Plan(cfg, max_hits=4096)
    cap_peaks, cap_pairs = 1 << 15, 1 << 19
    n_max = max(sum(e.n for e in evs) for evs in sets)
    bufs = H.BatchBuffers(plan, 3, n_max, cap_peaks, cap_pairs)
    refs = []
    for evs in sets:
        bufs.load(evs)
        bufs.run(cfg.threshold)
        torch.cuda.synchronize()
        refs.append([bufs.results(e) for e in range(3)])
    stream = torch.cuda.Stream()
    graph = H.Graph(bufs, cfg.threshold, stream)
    for rep in range(4):
        junk = torch.randn(1 << 18, device="cuda").sum()
        torch.cuda.synchronize()
        bufs.load(sets[rep % 2])
        bufs.zv.fill_(-9)
        bufs.status.fill_(-7)
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        for e in range(3):
            got, ref = bufs.results(e), refs[rep % 2][e]
            np.testing.assert_array_equal(got["peaks"], ref["peaks"])
            np.testing.assert_array_equal(got["zvote"], ref["zvote"])
        del junk
    graph.close()


def test_large_grid_batch_full_size_equals_oracle(H, oracle_mod):
    """The large-grid workload as benchmarked: a batch of 8 of its events (600 prompt tracks plus
    two displaced vertices, 20 % noise, with z) on the full 1024 x 512 x 128 int16 grid with the r-z
    stage, in one batched chain.  For every event: the whole accumulator and the whole candidate
    list equal the oracle's, every list length equals its candidate's votes, and sampled hit lists
    and r-z results equal the oracle's for those candidates."""
    O = oracle_mod
    cfg = configs.C4
    events = [synth.make_event(cfg, i) for i in range(8)]
    print(f"[zvote] full-size large-grid batch: hits {[e.n for e in events]}", flush=True)
    plan = H.Plan(cfg, max_hits=cfg.max_hits_per_event)
    # about 1.5M candidates and 1.2e7 pairs per event
    cap_peaks, cap_pairs = 1 << 21, 1 << 25
    bufs = H.BatchBuffers(plan, len(events), sum(e.n for e in events), cap_peaks, cap_pairs)
    bufs.load(events)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    g = O.Cfg(cfg)
    rng = np.random.default_rng(77)
    for e, ev in enumerate(events):
        got = bufs.results(e)
        st = got["status"]
        assert st["flags"] == 0, (e, st)
        acc_ref, nv = O.vote(g, ev)
        assert st["n_votes"] == nv
        acc = bufs.acc[e].to(torch.int32).cpu().numpy()
        np.testing.assert_array_equal(acc, acc_ref, err_msg=f"event {e} accumulator")
        del acc
        n, pk = O.peaks(g, acc_ref, cfg.threshold)
        del acc_ref
        assert st["n_peaks"] == n, e
        np.testing.assert_array_equal(got["peaks"], pk, err_msg=f"event {e} candidates")
        offs = got["offsets"]
        np.testing.assert_array_equal(np.diff(offs), pk[:, 3], err_msg=f"event {e} list lengths")
        assert st["n_pairs"] == int(pk[:, 3].sum())
        sel = np.unique(rng.choice(n, min(n, 300), replace=False))
        o_ref, h_ref, _ = O.assign(g, ev, pk[sel])
        for i, p in enumerate(sel):
            np.testing.assert_array_equal(got["hit_idx"][offs[p]:offs[p + 1]], h_ref[o_ref[i]:o_ref[i + 1]],
                                          err_msg=f"event {e} list of candidate {p}")
        z_ref = O.zvote(g, ev, pk[sel], o_ref, h_ref)
        np.testing.assert_array_equal(got["zvote"][sel], z_ref, err_msg=f"event {e} r-z")
        print(f"[zvote] event {e}: {ev.n} hits, {n} candidates, {st['n_pairs']} pairs equal the oracle", flush=True)
