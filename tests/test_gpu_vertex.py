"""Second transform (vertex space of the candidates): GPU against the CPU oracle through the C
ABI (hough_vertex_vote, hough_vertex_peaks).  Everything is integer, so the bar is equality:
the sample table entry by entry, the whole vertex accumulator and the vertex candidates."""
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


def _status(H, n_peaks):
    st = torch.zeros(H.STATUS_BYTES // 4, dtype=torch.int32, device="cuda")
    st[4] = int(n_peaks)  # n_peaks (int32 at byte 16)
    return st


def _gpu_vertex(H, vp, pk, cap, thr, n_peaks=None, cap_v=1 << 16):
    """Vertex vote and peaks of a host candidate list given to the GPU."""
    n_peaks = pk.shape[0] if n_peaks is None else n_peaks
    d_pk = torch.zeros((max(cap, 1), 4), dtype=torch.int32, device="cuda")
    if pk.shape[0]:
        d_pk[: pk.shape[0]] = torch.from_numpy(np.ascontiguousarray(pk[:cap], dtype=np.int32)).cuda()
    vb = H.VertexBuffers(vp, cap_peaks=max(cap, 1), cap_vpeaks=cap_v)
    vb.acc.fill_(-7)  # fully overwritten
    vb.run(d_pk, _status(H, n_peaks), thr)
    torch.cuda.synchronize()
    return vb.results()


def _oracle_vertex(O, cfg, vg, pk, thr):
    acc, nv = O.vertex_vote(O.Cfg(cfg), vg, pk)
    n, vpk = O.vertex_peaks(vg, acc, thr)
    return acc, nv, n, vpk


def _check(res, ref, n_given):
    acc, nv, n, vpk = ref
    np.testing.assert_array_equal(res["acc"], acc)
    st = res["status"]
    assert st["n_votes"] == nv == int(acc.sum())
    assert st["n_hits"] == n_given and st["n_peaks"] == n
    np.testing.assert_array_equal(res["peaks"], vpk)


def test_vertex_table_equals_oracle_samples(H, oracle_mod):
    """T[l][k][j] of the plan equals the oracle's sample at each row radius: every entry of a
    small grid, 20000 sampled entries of the large-grid workload's table."""
    O = oracle_mod
    for cfg, n_samples in ((configs.small_variant(configs.C4, n_phi=256, n_qpt=64, n_d0=8).with_(n_vr=64, n_vphi=64),
                            None), (configs.C4, 20000)):
        plan = H.Plan(cfg, max_hits=1024)
        vp = H.VertexPlan.of(plan)
        T = vp.table()
        g = O.Cfg(cfg)
        vg = O.VertexGrid.of(cfg)
        M = O.angle_bits(g)
        if n_samples is None:
            idx = np.argwhere(np.ones(T.shape, dtype=bool))
        else:
            rng = np.random.default_rng(5)
            idx = np.stack([rng.integers(0, n, n_samples) for n in T.shape], axis=1)
        bad = 0
        for l, k, j in idx:
            ok, E = O.sample(O.vertex_radius(vg, j), O.curvature(g, k), O.d0_centre(g, l), M)
            want = E if ok else -(1 << 31)
            bad += int(T[l, k, j] != want)
        assert bad == 0
        assert (T != -(1 << 31)).any() and (T == -(1 << 31)).any()


@pytest.mark.parametrize("n_vr,n_vphi,tracks,eid", [(64, 128, 30, 0), (128, 64, 60, 1), (64, 16, 8, 2),
                                                    (192, 256, 40, 3)])
def test_vertex_small_events_equal_oracle(H, oracle_mod, n_vr, n_vphi, tracks, eid):
    """The oracle's candidates of small LLP-search events (several rows slabs, a ragged last
    candidate range) through the GPU vertex stage."""
    O = oracle_mod
    cfg = configs.small_variant(configs.C4, n_tracks=tracks, n_phi=256, n_qpt=64, n_d0=8).with_(
        n_vr=n_vr, n_vphi=n_vphi, v_threshold=3)
    ev = synth.make_event(cfg, eid)
    g = O.Cfg(cfg)
    n, pk = O.peaks(g, O.vote(g, ev)[0], cfg.threshold)
    assert n > 10
    plan = H.Plan(cfg, max_hits=max(ev.n, 1))
    vp = H.VertexPlan.of(plan)
    vg = O.VertexGrid.of(cfg)
    ref = _oracle_vertex(O, cfg, vg, pk, cfg.v_threshold)
    assert ref[2] > 0
    _check(_gpu_vertex(H, vp, pk, n + 5, cfg.v_threshold), ref, n)


def test_vertex_launch_shapes_filter_and_caps(H, oracle_mod):
    """Any number of candidate ranges gives the same result (ranges of at most 65535 candidates
    are enforced); candidates below min_votes, beyond the capacity or outside the grid cast
    nothing; an empty list gives an empty space."""
    O = oracle_mod
    cfg = configs.small_variant(configs.C4, n_phi=256, n_qpt=64, n_d0=8).with_(n_vr=64, n_vphi=128)
    pk = synth.make_candidates(cfg, 150000, seed=11, votes=(5, 12))
    plan = H.Plan(cfg, max_hits=1024)
    vp = H.VertexPlan(plan, 64, 128, 0.0, 32.0, 8)
    vg = O.VertexGrid(64, 128, 0.0, 32.0, 8)
    ref = _oracle_vertex(O, cfg, vg, pk, 3)
    for groups in (1, 3, 64, 1000):
        vp.set_groups(groups)
        print(f"[vertex] groups={groups}", flush=True)
        _check(_gpu_vertex(H, vp, pk, pk.shape[0], 3), ref, pk.shape[0])
    vp.set_groups(17)
    # capacity below the count: the first cap candidates
    cap = 70001
    _check(_gpu_vertex(H, vp, pk, cap, 3, n_peaks=pk.shape[0]), _oracle_vertex(O, cfg, vg, pk[:cap], 3), cap)
    # bins outside the first grid are skipped
    bad = pk[:5000].copy()
    bad[::7, 0] = cfg.n_d0
    bad[1::7, 1] = -1
    bad[2::7, 2] = cfg.n_phi + 3
    good = np.ones(bad.shape[0], dtype=bool)
    good[::7] = good[1::7] = good[2::7] = False
    res = _gpu_vertex(H, vp, bad, bad.shape[0], 3)
    _check(res, _oracle_vertex(O, cfg, vg, bad[good], 3), bad.shape[0])
    # nothing listed
    res = _gpu_vertex(H, vp, pk[:0], 8, 1)
    assert not res["acc"].any() and res["status"]["n_votes"] == 0 and res["status"]["n_peaks"] == 0


def test_vertex_full_size_candidate_list(H, oracle_mod):
    """A candidate list of the large-grid workload's size (1.5 M bins of the 1024 x 512 x 128
    grid, votes 7..12), all voting, in the default launch shape: whole vertex space and vertex
    candidates equal the oracle's."""
    O = oracle_mod
    cfg = configs.C4
    pk = synth.make_candidates(cfg, 1500000, seed=1)
    plan = H.Plan(cfg, max_hits=1024)
    vp = H.VertexPlan.of(plan)
    vg = O.VertexGrid.of(cfg)
    print(f"[vertex] c4 full list groups={vp.groups}", flush=True)
    ref = _oracle_vertex(O, cfg, vg, pk, 3)
    _check(_gpu_vertex(H, vp, pk, 1 << 21, 3, cap_v=1 << 15), ref, pk.shape[0])


def test_vertex_after_gpu_chain_finds_llp_vertices(H, oracle_mod):
    """The device candidate list and status of the GPU chain feed the vertex stage directly.  On
    this clean event (the daughters of two displaced vertices only: 6 and 2 tracks) the result
    equals the oracle's chain and the fullest vertex candidate lies at the six-track vertex."""
    O = oracle_mod
    cfg = configs.C4.with_(n_tracks=0, noise_frac=0.0, v_threshold=2)
    ev = synth.make_event(cfg, 4)
    g = O.Cfg(cfg)
    n, pk = O.peaks(g, O.vote(g, ev)[0], cfg.threshold)
    plan = H.Plan(cfg, max_hits=1024)
    bufs = H.EventBuffers(plan, cap_peaks=1 << 12, cap_pairs=1 << 16)
    x, y, lay, _ = H.hits_to_device(ev)
    bufs.run(H.make_hits(x, y, lay), cfg.threshold, do_assign=False)
    vp = H.VertexPlan.of(plan)
    vb = H.VertexBuffers(vp, cap_peaks=1 << 12, cap_vpeaks=256)
    vb.run(bufs.peaks, bufs.status, cfg.v_threshold)
    torch.cuda.synchronize()
    res = vb.results()
    vg = O.VertexGrid.of(cfg)
    _check(res, _oracle_vertex(O, cfg, vg, pk, cfg.v_threshold), n)
    v = ev.truth["vertices"][0]
    assert (ev.truth["vertex"] == 0).sum() == 6
    jv = int(np.hypot(v[0], v[1]) / (cfg.vr_max - cfg.vr_min) * cfg.n_vr)
    bv = int((np.arctan2(v[1], v[0]) / (2 * np.pi)) % 1.0 * cfg.n_vphi)
    top = res["peaks"][np.argmax(res["peaks"][:, 3])]
    assert abs(int(top[1]) - jv) <= 1 and min((int(top[2]) - bv) % cfg.n_vphi, (bv - int(top[2])) % cfg.n_vphi) <= 1


def test_vertex_batch_equals_oracle(H, oracle_mod):
    """Several events at once (hough_vertex_vote_batch / hough_vertex_peaks_batch): uneven
    candidate counts, an event with no candidates and one whose count exceeds the capacity;
    every event equals the oracle's vertex space and vertex candidates."""
    O = oracle_mod
    cfg = configs.small_variant(configs.C4, n_phi=256, n_qpt=64, n_d0=8).with_(n_vr=128, n_vphi=64, v_threshold=3)
    lists = [synth.make_candidates(cfg, n, seed=20 + i) for i, n in enumerate((3000, 0, 800, 5000, 40))]
    cap = 4000
    n_ev = len(lists)
    plan = H.Plan(cfg, max_hits=1024)
    vp = H.VertexPlan.of(plan)
    vg = O.VertexGrid.of(cfg)
    pk = torch.zeros((n_ev, cap, 4), dtype=torch.int32, device="cuda")
    st = torch.zeros((n_ev, H.STATUS_BYTES // 4), dtype=torch.int32, device="cuda")
    for e, l in enumerate(lists):
        m = min(len(l), cap)
        if m:
            pk[e, :m] = torch.from_numpy(l[:m]).cuda()
        st[e, 4] = len(l)
    vb = H.VertexBatchBuffers(vp, n_ev, cap, 1 << 12)
    vb.acc.fill_(-5)
    vb.run(pk, st, cfg.v_threshold)
    torch.cuda.synchronize()
    for e, l in enumerate(lists):
        print(f"[vertex batch] event {e} candidates {len(l)}", flush=True)
        _check(vb.results(e), _oracle_vertex(O, cfg, vg, l[:cap], cfg.v_threshold), min(len(l), cap))


def test_vertex_batch_after_gpu_batch_chain(H, oracle_mod):
    """The batched first stage's device candidate lists and statuses feed the batched vertex stage
    directly; each event equals the oracle's chain."""
    O = oracle_mod
    cfg = configs.small_variant(configs.C4, n_tracks=25, n_phi=256, n_qpt=64, n_d0=8).with_(
        n_vr=64, n_vphi=128, v_threshold=3)
    events = [synth.make_event(cfg, i) for i in range(3)]
    plan = H.Plan(cfg, max_hits=1024)
    bufs = H.BatchBuffers(plan, len(events), sum(e.n for e in events), cap_peaks=1 << 13, cap_pairs=1 << 16)
    bufs.load(events)
    bufs.run(cfg.threshold, zvote=False)
    vp = H.VertexPlan.of(plan)
    vb = H.VertexBatchBuffers(vp, len(events), 1 << 13, 1 << 12)
    vb.run(bufs.peaks, bufs.status, cfg.v_threshold)
    torch.cuda.synchronize()
    g = O.Cfg(cfg)
    vg = O.VertexGrid.of(cfg)
    for e, ev in enumerate(events):
        n, pk = O.peaks(g, O.vote(g, ev)[0], cfg.threshold)
        _check(vb.results(e), _oracle_vertex(O, cfg, vg, pk, cfg.v_threshold), n)


def test_vertex_plan_rejects_unsupported_grids(H):
    """Vertex grids outside the stated limits are refused at plan time, with the documented code."""
    cfg = configs.small_variant(configs.C4, n_phi=256, n_qpt=64, n_d0=8)  # M = 8 + 7 = 15
    plan = H.Plan(cfg, max_hits=1024)
    bad = [((63, 64, 0.0, 32.0, 1), "unsupported"),     # rows not a multiple of 64
           ((64, 2048, 0.0, 32.0, 1), "unsupported"),   # more than 1024 azimuth bins
           ((64, 96, 0.0, 32.0, 1), "unsupported"),     # not a power of two
           ((64, 8, 0.0, 32.0, 1), "unsupported"),      # fewer than 16 bins
           ((64, 64, 5.0, 5.0, 1), "invalid"),          # empty radius range
           ((64, 64, -1.0, 32.0, 1), "invalid"),        # negative radius
           ((64, 64, 0.0, 32.0, 0), "invalid")]         # min_votes below 1
    for args, what in bad:
        with pytest.raises(H.HoughError, match=what):
            H.VertexPlan(plan, *args)
    vp = H.VertexPlan(plan, 128, 1024, 0.5, 40.0, 3)  # at the limits: accepted
    assert vp.groups >= 1
    with pytest.raises(H.HoughError, match="invalid"):
        vp.set_groups(0)
