"""The vote with each hit's own radius (hough_vote_cr: integer arcsine, every sample computed)
against the CPU oracle, bit for bit, on the paper's detector model (x/y smear); the unchanged peak
finder on its accumulator."""
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


def _run(H, cfg, ev, cap=1 << 16):
    plan = H.Plan(cfg, max_hits=max(ev.n, 1))
    acc = torch.full((cfg.n_d0, cfg.n_qpt, cfg.n_phi), -3, dtype=torch.int32, device="cuda")
    st = torch.zeros(H.STATUS_BYTES // 4, dtype=torch.int32, device="cuda")
    ws = torch.empty(plan.ws_bytes(cap), dtype=torch.uint8, device="cuda")
    pk = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
    x, y, lay, _ = H.hits_to_device(ev)
    H.vote_cr(plan, H.make_hits(x, y, lay), acc, st)
    H.peaks(plan, acc, cfg.threshold, pk, ws, st)
    torch.cuda.synchronize()
    s = H.status_dict(st)
    return acc.cpu().numpy(), s, pk[: min(s["n_peaks"], cap)].cpu().numpy()


def _check(H, O, cfg, ev):
    print(f"[cr] {cfg.name} n_hits={ev.n} grid={cfg.n_phi}x{cfg.n_qpt}x{cfg.n_d0}", flush=True)
    g = O.Cfg(cfg)
    acc, st, pk = _run(H, cfg, ev)
    ref, nv = O.vote_cr(g, ev)
    assert int(np.count_nonzero(acc != ref)) == 0
    assert st["n_votes"] == nv and st["n_hits"] == ev.n
    n, pk_ref = O.peaks(g, ref, cfg.threshold)
    assert st["n_peaks"] == n
    np.testing.assert_array_equal(pk, pk_ref)
    return st


@pytest.mark.parametrize("cfg,tracks,eid", [
    (configs.C7, 100, 0), (configs.C7.with_(n_qpt=64, n_phi=512), 300, 1), (configs.C6, 50, 2),
    (configs.C6.with_(n_d0=3, n_phi=16), 20, 3), (configs.C2.with_(n_phi=128, n_qpt=64, n_d0=8, smear_xy_cm=0.04), 40, 4)])
def test_cr_vote_equals_oracle(H, oracle_mod, cfg, tracks, eid):
    cfg = cfg.with_(n_tracks=tracks, n_events=1)
    _check(H, oracle_mod, cfg, synth.make_event(cfg, eid))


def test_cr_vote_full_size_paper_event(H, oracle_mod):
    """4000 curved prompt tracks (40 000 hits) on the paper's detector, 256 x 256 grid."""
    cfg = configs.C7.with_(n_tracks=4000)
    st = _check(H, oracle_mod, cfg, synth.make_event(cfg, 0))
    assert st["n_votes"] > 5_000_000


def test_cr_vote_bad_and_empty(H, oracle_mod):
    cfg = configs.C7.with_(n_tracks=30)
    ev = synth.make_event(cfg, 5)
    x, y, lay = ev.x.copy(), ev.y.copy(), ev.layer.copy()
    x[0] = np.nan
    y[1] = 40000.0
    lay[2] = 12
    x[3] = y[3] = 0.0
    bad = synth.Event(x=x, y=y, z=None, layer=lay, track_id=ev.track_id, truth=ev.truth)
    st = _check(H, oracle_mod, cfg, bad)
    assert st["n_bad_hits"] == 4
    empty = synth.Event(x=np.zeros(0, np.float32), y=np.zeros(0, np.float32), z=None,
                        layer=np.zeros(0, np.uint8), track_id=np.zeros(0, np.int32), truth={})
    acc, st, pk = _run(H, cfg, empty)
    assert not acc.any() and st["n_votes"] == 0 and st["n_peaks"] == 0


def test_cr_rejects_int16_accumulator(H):
    cfg = configs.C4
    plan = H.Plan(cfg, max_hits=1024)
    ev = synth.make_event(configs.C7.with_(n_tracks=2), 0)
    x, y, lay, _ = H.hits_to_device(ev)
    acc = torch.zeros(4, dtype=torch.int32, device="cuda")
    st = torch.zeros(H.STATUS_BYTES // 4, dtype=torch.int32, device="cuda")
    with pytest.raises(H.HoughError, match="unsupported"):
        H.vote_cr(plan, H.make_hits(x, y, lay), acc, st)


def _run_assign(H, cfg, ev, cap_peaks=1 << 16, cap_pairs=1 << 22):
    """vote_cr -> peaks -> assign_cr -> fit on the GPU; returns (status, candidates, offsets, lists, fit)."""
    plan = H.Plan(cfg, max_hits=max(ev.n, 1))
    acc = torch.empty((cfg.n_d0, cfg.n_qpt, cfg.n_phi), dtype=torch.int32, device="cuda")
    st = torch.zeros(H.STATUS_BYTES // 4, dtype=torch.int32, device="cuda")
    ws = torch.empty(plan.ws_bytes(cap_peaks), dtype=torch.uint8, device="cuda")
    ws_cr = torch.empty(H.assign_cr_ws_bytes(plan, cap_peaks, cap_pairs), dtype=torch.uint8, device="cuda")
    pk = torch.empty((cap_peaks, 4), dtype=torch.int32, device="cuda")
    offs = torch.full((cap_peaks + 1,), -7, dtype=torch.int32, device="cuda")
    hit_idx = torch.full((cap_pairs,), -7, dtype=torch.int32, device="cuda")
    x, y, lay, _ = H.hits_to_device(ev)
    hits = H.make_hits(x, y, lay)
    H.vote_cr(plan, hits, acc, st)
    H.peaks(plan, acc, cfg.threshold, pk, ws, st)
    H.assign_cr(plan, hits, pk, offs, hit_idx, ws, ws_cr, st)
    fit = torch.full((cap_peaks, 4), 7.0, dtype=torch.float64, device="cuda")
    H.fit(plan, hits, offs, hit_idx, st, fit)
    torch.cuda.synchronize()
    s = H.status_dict(st)
    n = min(s["n_peaks"], cap_peaks)
    return (s, pk[:n].cpu().numpy(), offs[: n + 1].cpu().numpy().astype(np.int64),
            hit_idx[: min(s["n_pairs"], cap_pairs)].cpu().numpy(), fit[:n].cpu().numpy())


@pytest.mark.parametrize("cfg,tracks,eid", [
    (configs.C7, 100, 10), (configs.C6, 50, 11), (configs.C7.with_(n_qpt=64, n_phi=512), 300, 12),
    (configs.C2.with_(n_phi=128, n_qpt=64, n_d0=8, smear_xy_cm=0.04), 40, 13)])
def test_cr_assign_equals_oracle(H, oracle_mod, cfg, tracks, eid):
    """Lists of every candidate of a per-hit-radius accumulator, and their fits, equal the oracle's."""
    O = oracle_mod
    cfg = cfg.with_(n_tracks=tracks, n_events=1)
    ev = synth.make_event(cfg, eid)
    print(f"[cr-assign] {cfg.name} n_hits={ev.n}", flush=True)
    st, pk, offs, hit_idx, fit = _run_assign(H, cfg, ev)
    g = O.Cfg(cfg)
    ref, _ = O.vote_cr(g, ev)
    n, pk_ref = O.peaks(g, ref, cfg.threshold)
    np.testing.assert_array_equal(pk, pk_ref)
    o_ref, h_ref, tot = O.assign_cr(g, ev, pk_ref)
    assert st["n_pairs"] == tot and st["flags"] == 0
    np.testing.assert_array_equal(offs, o_ref)
    np.testing.assert_array_equal(hit_idx, h_ref)
    np.testing.assert_array_equal(fit, O.fit(ev, o_ref, h_ref))


def test_cr_assign_full_size_and_cut(H, oracle_mod):
    """The 4000-track paper-detector event: 300 sampled lists equal the oracle's; then with a pair
    capacity that cuts the lists, the kept entries are the same and the cut is flagged."""
    O = oracle_mod
    cfg = configs.C7.with_(n_tracks=4000)
    ev = synth.make_event(cfg, 0)
    print(f"[cr-assign] full size n_hits={ev.n}", flush=True)
    st, pk, offs, hit_idx, _ = _run_assign(H, cfg, ev, cap_pairs=1 << 24)
    g = O.Cfg(cfg)
    n = pk.shape[0]
    assert st["flags"] == 0 and st["n_pairs"] == int(pk[:, 3].sum()) and n > 1000
    np.testing.assert_array_equal(np.diff(offs), pk[:, 3])
    sel = np.unique(np.random.default_rng(5).choice(n, 300, replace=False))
    o_ref, h_ref, _ = O.assign_cr(g, ev, pk[sel])
    for i, p in enumerate(sel):
        np.testing.assert_array_equal(hit_idx[offs[p]:offs[p + 1]], h_ref[o_ref[i]:o_ref[i + 1]], err_msg=str(p))
    cap = int(st["n_pairs"] // 3) + 5
    st2, pk2, offs2, hit2, fit2 = _run_assign(H, cfg, ev, cap_pairs=cap)
    assert st2["flags"] & 2 and st2["n_pairs"] == st["n_pairs"]
    np.testing.assert_array_equal(offs2, offs)
    np.testing.assert_array_equal(hit2, hit_idx[:cap])
    assert (fit2[offs2[1:] > cap, 2] == -2.0).all()
