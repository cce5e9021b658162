"""GPU path (libhough.so through its C ABI) against the CPU oracle.

Bit-exact comparisons throughout (integer work: accumulators, candidate lists,
CSR hit lists, azimuths): the tolerance is zero.  Small grids are compared in
full; the full-size workloads are compared in full where the oracle finishes in
seconds, otherwise on sampled columns/candidates.
"""
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


def _event(x, y, layer, z=None):
    n = len(x)
    return synth.Event(x=np.asarray(x, np.float32), y=np.asarray(y, np.float32),
                       z=None if z is None else np.asarray(z, np.float32), layer=np.asarray(layer, np.uint8),
                       track_id=np.full(n, -1, np.int32), truth={})


def run_gpu(H, cfg, ev, cap_peaks=1 << 18, cap_pairs=1 << 22, max_hits=None, plan=None):
    plan = plan or H.Plan(cfg, max_hits=max_hits or max(ev.n, 1))
    bufs = H.EventBuffers(plan, cap_peaks=cap_peaks, cap_pairs=cap_pairs)
    x, y, lay, _ = H.hits_to_device(ev)
    bufs.run(H.make_hits(x, y, lay), cfg.threshold)
    torch.cuda.synchronize()
    res = bufs.results()
    res["acc"] = bufs.acc.cpu().numpy().astype(np.int32)
    return res


def check_full(H, O, cfg, ev, **kw):
    print(f"[parity] {cfg.name} n_hits={ev.n}", flush=True)
    g = O.Cfg(cfg)
    res = run_gpu(H, cfg, ev, **kw)
    acc_ref, nv = O.vote(g, ev)
    assert res["status"]["n_votes"] == nv
    mism = int(np.count_nonzero(res["acc"] != acc_ref))
    assert mism == 0, f"{mism} accumulator mismatches"
    n_ref, pk_ref = O.peaks(g, acc_ref, cfg.threshold)
    assert res["status"]["n_peaks"] == n_ref
    np.testing.assert_array_equal(res["peaks"], pk_ref)
    offs_ref, hit_ref, tot = O.assign(g, ev, pk_ref)
    assert res["status"]["n_pairs"] == tot
    np.testing.assert_array_equal(res["offsets"], offs_ref)
    np.testing.assert_array_equal(res["hit_idx"], hit_ref)
    return res, acc_ref, pk_ref


# ----------------------------------------------------------------- prep --
def test_prep_azimuth_bit_exact(H, oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(21)
    n = 5000
    r = 10 ** rng.uniform(-1, 4.3, n)
    phi = rng.uniform(0, 2 * np.pi, n)
    x = (r * np.cos(phi)).astype(np.float32)
    y = (r * np.sin(phi)).astype(np.float32)
    lay = rng.integers(0, 10, n).astype(np.uint8)
    # edge cases: non-finite, out of range, bad layer, origin, axes, ties of the Q16.16 rounding
    x[:12] = [np.nan, np.inf, 40000.0, 5.0, 0.0, 2 ** -18, 1.0, 0.0, -1.0, 0.0, 1.5 / 65536, 32767.0]
    y[:12] = [1.0, 1.0, 1.0, 5.0, 0.0, 0.0, 0.0, 1.0, 0.0, -1.0, 2.5 / 65536, -32767.0]
    lay[3] = 10
    ev = _event(x, y, lay)
    cfg = configs.C2
    plan = H.Plan(cfg, max_hits=n)
    ws = torch.empty(plan.ws_bytes(), dtype=torch.uint8, device="cuda")
    st = torch.zeros(8, dtype=torch.int32, device="cuda")
    phi_out = torch.empty(n, dtype=torch.int32, device="cuda")
    xd, yd, ld, _ = H.hits_to_device(ev)
    H.prep(plan, H.make_hits(xd, yd, ld), phi_out, ws, st)
    torch.cuda.synchronize()
    got = phi_out.cpu().numpy().view(np.uint32)
    want, ok = O.prep(ev, 10)
    np.testing.assert_array_equal(got, want)
    assert H.status_dict(st)["n_bad_hits"] == int((~ok).sum())
    assert H.status_dict(st)["n_bad_hits"] >= 6


def test_plan_table_matches_oracle_samples(H, oracle_mod):
    O = oracle_mod
    for cfg in (configs.C1, configs.C2, configs.C4):
        plan = H.Plan(cfg, max_hits=100)
        tab = plan.table()
        g = O.Cfg(cfg)
        M = O.angle_bits(g)
        assert plan.angle_bits == M
        rng = np.random.default_rng(cfg.cfg_id)
        for _ in range(4000):
            L = int(rng.integers(0, 10)); l = int(rng.integers(0, cfg.n_d0)); k = int(rng.integers(0, cfg.n_qpt))
            ok, E = O.sample(cfg.radii_cm[L], O.curvature(g, k), O.d0_centre(g, l), M)
            assert tab[L, l, k] == (E if ok else np.iinfo(np.int32).min)


# ----------------------------------------------------------- full parity --
@pytest.mark.parametrize("event_id", [0, 1, 2])
def test_c1_full_parity(H, oracle_mod, event_id):
    check_full(H, oracle_mod, configs.C1, synth.make_event(configs.C1, event_id))


@pytest.mark.parametrize("shape,tracks,eid,frac", [
    ((512, 64, 8), 30, 0, 7), ((512, 128, 16), 57, 1, 7), ((256, 64, 3), 11, 2, 7), ((512, 64, 5), 45, 3, 7),
    ((128, 192, 7), 23, 4, 7), ((16, 64, 2), 5, 5, 7), ((1024, 64, 4), 40, 6, 7),
    ((512, 64, 8), 30, 0, 8), ((256, 128, 5), 33, 7, 8), ((16, 64, 3), 6, 8, 8)])
def test_c2_family_small_full_parity(H, oracle_mod, shape, tracks, eid, frac):
    """frac_bits 7: 16-bit vote counters in LDS, int32 accumulator; 8: 32-bit counters."""
    nphi, nqpt, nd0 = shape
    cfg = configs.small_variant(configs.C2, n_tracks=tracks, n_phi=nphi, n_qpt=nqpt, n_d0=nd0).with_(frac_bits=frac)
    check_full(H, oracle_mod, cfg, synth.make_event(cfg, eid))


@pytest.mark.parametrize("cfg,tracks", [(configs.C6, 50), (configs.C7, 300)])
def test_paper_detector_full_parity(H, oracle_mod, cfg, tracks):
    """The paper's own detector (layers at 11..110 cm, 0.4 mm x/y smear): the 50 straight lines of
    its first figure (B = 0: every q/pT row holds the same line space) and curved prompt tracks in
    the two-parameter space."""
    cfg = cfg.with_(n_tracks=tracks)
    check_full(H, oracle_mod, cfg, synth.make_event(cfg, 0))


def test_c4_family_int16_small_full_parity(H, oracle_mod):
    cfg = configs.small_variant(configs.C4, n_tracks=60, n_phi=1024, n_qpt=64, n_d0=6)
    ev = synth.make_event(cfg, 0)
    check_full(H, oracle_mod, cfg, ev)


def test_c2_full_size_parity(H, oracle_mod):
    """The full dense event (about 12k hits, 512x256x64 bins) in the tuned launch
    shape: accumulator and candidate list compared in full, hit lists on sampled
    candidates plus the first and last ones, CSR offsets in full."""
    O = oracle_mod
    cfg = configs.C2
    ev = synth.make_event(cfg, 0)
    print(f"[parity] c2 full n_hits={ev.n}", flush=True)
    g = O.Cfg(cfg)
    from paper_1305_4855_amd import tune
    plan = H.Plan(cfg, max_hits=16384)
    print(f"[parity] c2 full launch shape {tune.apply(plan)}", flush=True)  # the benchmark's shape
    res = run_gpu(H, cfg, ev, cap_peaks=1 << 19, cap_pairs=1 << 24, plan=plan)
    acc_ref, nv = O.vote(g, ev)
    assert int(np.count_nonzero(res["acc"] != acc_ref)) == 0
    assert res["status"]["n_votes"] == nv
    n_ref, pk_ref = O.peaks(g, acc_ref, cfg.threshold)
    assert res["status"]["n_peaks"] == n_ref
    np.testing.assert_array_equal(res["peaks"], pk_ref)
    offs = res["offsets"]
    np.testing.assert_array_equal(np.diff(offs), pk_ref[:, 3])
    assert offs[0] == 0 and res["status"]["n_pairs"] == int(pk_ref[:, 3].sum())
    rng = np.random.default_rng(22)
    sel = np.unique(np.concatenate([np.arange(50), np.arange(n_ref - 50, n_ref),
                                    rng.choice(n_ref, 400, replace=False)]))
    offs_s, hit_s, _ = O.assign(g, ev, pk_ref[sel])
    for j, p in enumerate(sel):
        np.testing.assert_array_equal(res["hit_idx"][offs[p]:offs[p + 1]], hit_s[offs_s[j]:offs_s[j + 1]])


def test_c4_full_size_vote_parity(H, oracle_mod):
    """Full LLP-search grid (1024x512x128, int16): accumulator in full."""
    O = oracle_mod
    cfg = configs.C4
    ev = synth.make_event(cfg, 0)
    print(f"[parity] c4 full n_hits={ev.n}", flush=True)
    plan = H.Plan(cfg, max_hits=16384)
    acc = torch.empty((cfg.n_d0, cfg.n_qpt, cfg.n_phi), dtype=torch.int16, device="cuda")
    ws = torch.empty(plan.ws_bytes(), dtype=torch.uint8, device="cuda")
    st = torch.zeros(8, dtype=torch.int32, device="cuda")
    x, y, lay, _ = H.hits_to_device(ev)
    H.vote(plan, H.make_hits(x, y, lay), acc, ws, st)
    torch.cuda.synchronize()
    got = acc.cpu().numpy()
    rng = np.random.default_rng(23)
    cols = np.stack([rng.integers(0, cfg.n_d0, 256), rng.integers(0, cfg.n_qpt, 256)], axis=1)
    want = O.vote_columns(O.Cfg(cfg), ev, cols)
    np.testing.assert_array_equal(got[cols[:, 0], cols[:, 1]].astype(np.int32), want)
    acc_ref, nv = O.vote(O.Cfg(cfg), ev)
    assert H.status_dict(st)["n_votes"] == nv
    assert int(np.count_nonzero(got.astype(np.int32) != acc_ref)) == 0


# ------------------------------------------------------------ edge cases --
def test_empty_event(H, oracle_mod):
    cfg = configs.small_variant(configs.C2, n_phi=256, n_qpt=64, n_d0=4)
    ev = _event([], [], [])
    res = run_gpu(H, cfg, ev, max_hits=16)
    assert not res["acc"].any()
    assert res["status"]["n_peaks"] == 0 and res["status"]["n_pairs"] == 0 and res["status"]["n_votes"] == 0


def test_single_hit_and_bad_hits(H, oracle_mod):
    cfg = configs.small_variant(configs.C2, n_phi=256, n_qpt=64, n_d0=4).with_(threshold=1)
    ev = _event([10.2, np.nan, 0.0, 5.0, 1e6], [0.0, 1.0, 0.0, 5.0, 1.0], [2, 2, 2, 11, 3])
    res, _, _ = check_full(H, oracle_mod, cfg, ev, max_hits=8)
    assert res["status"]["n_bad_hits"] == 4


def test_ragged_hit_counts(H, oracle_mod):
    """Hit counts around the 64-hit chunk and 16-wave boundaries of the vote."""
    cfg = configs.small_variant(configs.C2, n_phi=256, n_qpt=64, n_d0=4).with_(threshold=2)
    rng = np.random.default_rng(24)
    r = np.asarray(configs.RADII_CM)
    for n in (1, 63, 64, 65, 1023, 1024, 1025, 2049):
        lay = np.zeros(n, np.uint8) if n < 100 else rng.integers(0, 10, n).astype(np.uint8)
        phi = rng.uniform(0, 2 * np.pi, n)
        ev = _event(r[lay] * np.cos(phi), r[lay] * np.sin(phi), lay)
        check_full(H, oracle_mod, cfg, ev, max_hits=n)


def test_bucket_sort_limit_and_crowded_cells(H, oracle_mod):
    """Events at and just past the size the bucketing workgroup sorts in its LDS (16384 hits;
    larger ones go through the separate rank pass), with crowded cells (more than 8 hits, the
    in-cell ranking's first round) and hits at identical angles (ties broken by hit index); alone
    against the oracle, and mixed in one batch against the single-event path."""
    cfg = configs.small_variant(configs.C2, n_phi=256, n_qpt=64, n_d0=2).with_(threshold=30)
    rng = np.random.default_rng(26)
    r = np.asarray(configs.RADII_CM)

    def event(n):
        lay = rng.integers(0, 10, n).astype(np.uint8)
        phi = rng.uniform(0, 2 * np.pi, n)
        phi[: n // 8] = rng.uniform(1.0, 1.02, n // 8)  # crowded cells
        phi[n // 8: n // 8 + 40] = 2.5                    # identical angles
        lay[n // 8: n // 8 + 40] = 3
        return _event(r[lay] * np.cos(phi), r[lay] * np.sin(phi), lay)

    events = [event(n) for n in (16383, 16384, 16385)]
    for ev in events:
        check_full(H, oracle_mod, cfg, ev, max_hits=20000, cap_peaks=1 << 16, cap_pairs=1 << 23)
    plan = H.Plan(cfg, max_hits=20000)
    mixed = [events[2], events[0], synth.make_event(cfg.with_(n_tracks=20, track_dist="fixed"), 5), events[1]]
    bufs = H.BatchBuffers(plan, len(mixed), sum(e.n for e in mixed), 1 << 16, 1 << 23)
    bufs.load(mixed)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    for e, ev in enumerate(mixed):
        single = run_gpu(H, cfg, ev, cap_peaks=1 << 16, cap_pairs=1 << 23, plan=plan)
        got = bufs.results(e)
        np.testing.assert_array_equal(got["peaks"], single["peaks"])
        np.testing.assert_array_equal(got["hit_idx"], single["hit_idx"])


def test_large_events_take_the_long_paths(H, oracle_mod):
    """Events beyond what the fast paths hold: more hits than the bucketing keeps in registers
    (16384), more valid hits than the assignment stages in LDS, more than 65535 hits with 32-bit
    vote counters (frac_bits 8), and a batch mixing such an event with small ones."""
    cfg = configs.small_variant(configs.C2, n_phi=256, n_qpt=64, n_d0=2).with_(threshold=30)
    rng = np.random.default_rng(25)
    r = np.asarray(configs.RADII_CM)
    for n, frac in ((30000, 7), (65535, 7), (70000, 8)):
        lay = rng.integers(0, 10, n).astype(np.uint8)
        phi = rng.uniform(0, 2 * np.pi, n)
        ev = _event(r[lay] * np.cos(phi), r[lay] * np.sin(phi), lay)
        check_full(H, oracle_mod, cfg.with_(frac_bits=frac), ev, max_hits=n, cap_peaks=1 << 16, cap_pairs=1 << 23)
    n = 30000
    lay = rng.integers(0, 10, n).astype(np.uint8)
    phi = rng.uniform(0, 2 * np.pi, n)
    big = _event(r[lay] * np.cos(phi), r[lay] * np.sin(phi), lay)
    small = [synth.make_event(cfg.with_(n_tracks=t, track_dist="fixed"), 40 + i) for i, t in enumerate([3, 50])]
    events = [small[0], big, small[1]]
    plan = H.Plan(cfg, max_hits=n)
    bufs = H.BatchBuffers(plan, 3, sum(e.n for e in events), 1 << 16, 1 << 23)
    bufs.load(events)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    for e, ev in enumerate(events):
        single = run_gpu(H, cfg, ev, cap_peaks=1 << 16, cap_pairs=1 << 23, plan=plan)
        got = bufs.results(e)
        np.testing.assert_array_equal(got["peaks"], single["peaks"])
        np.testing.assert_array_equal(got["hit_idx"], single["hit_idx"])
        np.testing.assert_array_equal(bufs.acc[e].cpu().numpy(), single["acc"])


def test_capacity_overflow(H, oracle_mod):
    O = oracle_mod
    cfg = configs.small_variant(configs.C2, n_tracks=40, n_phi=256, n_qpt=64, n_d0=8)
    ev = synth.make_event(cfg, 7)
    g = O.Cfg(cfg)
    acc_ref, _ = O.vote(g, ev)
    n_ref, pk_ref = O.peaks(g, acc_ref, cfg.threshold)
    assert n_ref > 20
    res = run_gpu(H, cfg, ev, cap_peaks=17, cap_pairs=50)
    st = res["status"]
    assert st["n_peaks"] == n_ref and st["flags"] & H.HOUGH_F_PEAK_OVERFLOW
    np.testing.assert_array_equal(res["peaks"], pk_ref[:17])
    offs_ref, hit_ref, tot = O.assign(g, ev, pk_ref[:17])
    assert st["n_pairs"] == tot and (st["flags"] & H.HOUGH_F_PAIR_OVERFLOW) == (H.HOUGH_F_PAIR_OVERFLOW if tot > 50 else 0)
    np.testing.assert_array_equal(res["offsets"], offs_ref)
    np.testing.assert_array_equal(res["hit_idx"], hit_ref[:50])


def test_unsupported_grids_rejected(H):
    # a vote slab of 64 columns x 1024 phi0 bins of 32-bit counters (frac_bits 8), or of 2048
    # bins of 16-bit counters (frac_bits 7), needs 256 KiB of LDS (160 KiB on gfx950)
    with pytest.raises(H.HoughError, match="unsupported"):
        H.Plan(configs.C2.with_(n_phi=1024, frac_bits=8), max_hits=10)
    with pytest.raises(H.HoughError, match="unsupported"):
        H.Plan(configs.C2.with_(n_phi=2048), max_hits=10)
    # 16-bit counters: at most 65535 hits per event (32767 for an int16 accumulator)
    with pytest.raises(H.HoughError, match="unsupported"):
        H.Plan(configs.C2, max_hits=65536)
    with pytest.raises(H.HoughError, match="unsupported"):
        H.Plan(configs.C2.with_(frac_bits=6), max_hits=10)
    with pytest.raises(H.HoughError, match="unsupported"):
        H.Plan(configs.C2.with_(n_qpt=100), max_hits=10)
    with pytest.raises(H.HoughError, match="unsupported"):
        H.Plan(configs.C2.with_(n_phi=500), max_hits=10)
    with pytest.raises(H.HoughError, match="unsupported"):
        H.Plan(configs.C4.with_(max_hits_per_event=40000), max_hits=40000)


def test_too_many_hits_rejected(H):
    cfg = configs.small_variant(configs.C2, n_phi=256, n_qpt=64, n_d0=4)
    plan = H.Plan(cfg, max_hits=10)
    x = torch.zeros(11, dtype=torch.float32, device="cuda")
    lay = torch.zeros(11, dtype=torch.uint8, device="cuda")
    acc = torch.empty(plan.acc_bytes // 4, dtype=torch.int32, device="cuda")
    ws = torch.empty(plan.ws_bytes(), dtype=torch.uint8, device="cuda")
    st = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(H.HoughError):
        H.vote(plan, H.make_hits(x, x, lay), acc, ws, st)


def test_deterministic_and_rotation_covariant(H):
    cfg = configs.small_variant(configs.C2, n_tracks=50, n_phi=512, n_qpt=64, n_d0=8)
    ev = synth.make_event(cfg, 9)
    a = run_gpu(H, cfg, ev)
    b = run_gpu(H, cfg, ev)
    for key in ("acc", "peaks", "offsets", "hit_idx"):
        np.testing.assert_array_equal(a[key], b[key])
    rot = _event(-ev.y, ev.x, ev.layer)
    c = run_gpu(H, cfg, rot)
    np.testing.assert_array_equal(np.roll(a["acc"], cfg.n_phi // 4, axis=2), c["acc"])
