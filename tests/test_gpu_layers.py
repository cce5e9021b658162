"""Detectors with more layers than the kernels take in one group (ten): the table vote reads the
samples and window counts of layers 10.. in further groups, and so does the assignment.  A
13-layer and a 32-layer (the largest supported) detector, single events and a batch (the batch
reads the 8-bit window counts), against the CPU oracle, bit-exact."""
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


def _cfg(n_layers):
    radii = tuple(float(r) for r in np.linspace(4.4, 110.0, n_layers))
    base = configs.small_variant(configs.C3, n_tracks=30, n_phi=256, n_qpt=64, n_d0=8)
    return base.with_(name=f"c3_small_{n_layers}_layers", radii_cm=radii, halflen_cm=(110.0,) * n_layers)


def _check(O, cfg, ev, acc, res, ctx):
    g = O.Cfg(cfg)
    acc_ref, nv = O.vote(g, ev)
    assert int(np.count_nonzero(acc != acc_ref)) == 0, f"{ctx}: accumulator"
    assert res["status"]["n_votes"] == nv, ctx
    n_ref, pk_ref = O.peaks(g, acc_ref, cfg.threshold)
    assert res["status"]["n_peaks"] == n_ref, ctx
    np.testing.assert_array_equal(res["peaks"], pk_ref, err_msg=ctx)
    offs_ref, hit_ref, tot = O.assign(g, ev, pk_ref)
    assert res["status"]["n_pairs"] == tot, ctx
    np.testing.assert_array_equal(res["offsets"], offs_ref, err_msg=ctx)
    np.testing.assert_array_equal(res["hit_idx"], hit_ref, err_msg=ctx)


@pytest.mark.parametrize("n_layers", [13, 32])
def test_single_event_many_layers_equals_oracle(H, oracle_mod, n_layers):
    cfg = _cfg(n_layers)
    ev = synth.make_event(cfg, 0)
    print(f"[layers] single {n_layers} layers, {ev.n} hits", flush=True)
    plan = H.Plan(cfg, max_hits=max(ev.n, 1))
    bufs = H.EventBuffers(plan, cap_peaks=1 << 16, cap_pairs=1 << 20)
    x, y, lay, _ = H.hits_to_device(ev)
    bufs.run(H.make_hits(x, y, lay), cfg.threshold)
    torch.cuda.synchronize()
    res = bufs.results()
    _check(oracle_mod, cfg, ev, bufs.acc.cpu().numpy().astype(np.int32), res, f"{n_layers} layers")


@pytest.mark.parametrize("n_layers", [13, 32])
def test_batch_many_layers_equals_oracle(H, oracle_mod, n_layers):
    cfg = _cfg(n_layers)
    events = [synth.make_event(cfg.with_(n_tracks=nt, track_dist="fixed"), i) for i, nt in enumerate([30, 5, 50])]
    print(f"[layers] batch {n_layers} layers, {[e.n for e in events]} hits", flush=True)
    plan = H.Plan(cfg, max_hits=4096)
    bufs = H.BatchBuffers(plan, len(events), sum(e.n for e in events), 1 << 16, 1 << 20)
    bufs.load(events)
    bufs.run(cfg.threshold)
    torch.cuda.synchronize()
    acc = bufs.acc.cpu().numpy()
    for e, ev in enumerate(events):
        _check(oracle_mod, cfg, ev, acc[e].astype(np.int32), bufs.results(e), f"{n_layers} layers, event {e}")
