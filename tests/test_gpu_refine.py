"""Background suppression inside each candidate's bin (hough_refine) against the oracle: for every
candidate, the refined hit of each layer and the number of layers, bit for bit."""
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


def _gpu_refine(H, cfg, ev, window, cap_peaks=1 << 19, cap_pairs=1 << 24, max_hits=None):
    plan = H.Plan(cfg, max_hits=max_hits or max(ev.n, 16))
    bufs = H.EventBuffers(plan, cap_peaks=cap_peaks, cap_pairs=cap_pairs)
    x, y, lay, _ = H.hits_to_device(ev)
    bufs.run(H.make_hits(x, y, lay), cfg.threshold)
    out_h = torch.full((cap_peaks, cfg.n_layers), -9, dtype=torch.int32, device="cuda")
    out_l = torch.full((cap_peaks,), -9, dtype=torch.int32, device="cuda")
    H.refine(plan, bufs.peaks, bufs.offsets, bufs.hit_idx, bufs.ws, bufs.status, window, out_h, out_l)
    torch.cuda.synchronize()
    r = bufs.results()
    n = r["peaks"].shape[0]
    return r, out_h[:n].cpu().numpy(), out_l[:n].cpu().numpy()


@pytest.mark.parametrize("cfg,tracks,eid,window", [
    (configs.C7, 500, 0, 16), (configs.C7, 60, 1, 4), (configs.C7.with_(n_phi=512, n_qpt=64), 300, 2, 128),
    (configs.small_variant(configs.C2, n_tracks=60, n_phi=256, n_qpt=64, n_d0=8), 60, 3, 16)])
def test_refine_equals_oracle(H, oracle_mod, cfg, tracks, eid, window):
    O = oracle_mod
    cfg = cfg.with_(n_tracks=tracks, n_events=1)
    ev = synth.make_event(cfg, eid)
    print(f"[refine] {cfg.name} n_hits={ev.n} window={window}", flush=True)
    r, gh, gl = _gpu_refine(H, cfg, ev, window)
    g = O.Cfg(cfg)
    acc, _ = O.vote(g, ev)
    n, pk = O.peaks(g, acc, cfg.threshold)
    np.testing.assert_array_equal(r["peaks"], pk)
    offs, hit_idx, _ = O.assign(g, ev, pk)
    oh, ol = O.refine(g, ev, pk, offs, hit_idx, window)
    np.testing.assert_array_equal(gl, ol)
    np.testing.assert_array_equal(gh, oh)
    assert (gl > 0).any()


@pytest.mark.parametrize("cfg,long_lists", [
    (configs.C2, False),
    (configs.C7.with_(n_phi=128, n_qpt=64, n_tracks=4000), True)])
def test_refine_dense_event_and_cut_lists(H, oracle_mod, cfg, long_lists):
    """Every candidate of a dense event (the 512x256x64 single event; a coarse 128x64 grid of 4000
    paper-detector tracks, whose lists exceed the LDS stage), then the same event with a pair
    capacity that cuts the lists: cut lists report -1, the others are unchanged."""
    O = oracle_mod
    ev = synth.make_event(cfg, 0)
    print(f"[refine-dense] {cfg.name} n_hits={ev.n} grid={cfg.n_phi}x{cfg.n_qpt}x{cfg.n_d0}", flush=True)
    r, gh, gl = _gpu_refine(H, cfg, ev, 16, max_hits=max(16384, ev.n))
    g = O.Cfg(cfg)
    pk = r["peaks"]
    assert (int(pk[:, 3].max()) > 64) == long_lists  # lists past the LDS stage take the unstaged path
    oh, ol = O.refine(g, ev, pk, r["offsets"], r["hit_idx"], 16)
    np.testing.assert_array_equal(gl, ol)
    np.testing.assert_array_equal(gh, oh)
    cap = int(r["status"]["n_pairs"] // 2)
    r2, gh2, gl2 = _gpu_refine(H, cfg, ev, 16, cap_pairs=cap, max_hits=max(16384, ev.n))
    cut = r2["offsets"][1:] > cap
    assert cut.any() and (gl2[cut] == -1).all() and (gh2[cut] == -1).all()
    np.testing.assert_array_equal(gl2[~cut], ol[~cut])
    np.testing.assert_array_equal(gh2[~cut], oh[~cut])
