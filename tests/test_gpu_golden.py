"""The GPU chain on the small single-event workload against the stored
expected values in tests/golden/ (written from the CPU oracle)."""
import numpy as np
import pytest

from paper_1305_4855_amd import configs, synth
from tests.golden_io import read_c1_event0

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_4855_amd import hough as H
    return H


def _check(res, gold):
    assert res["status"]["n_votes"] == gold["votes"]
    assert res["status"]["n_peaks"] == gold["candidates"]
    assert res["status"]["n_pairs"] == gold["pairs"]
    np.testing.assert_array_equal(res["peaks"], gold["cands"])
    offs = res["offsets"]
    for i, lst in enumerate(gold["lists"]):
        assert list(res["hit_idx"][offs[i]:offs[i + 1]]) == lst


def test_c1_event0_single_and_batch(H):
    gold = read_c1_event0()
    cfg = configs.C1
    ev = synth.make_event(cfg, 0)
    plan = H.Plan(cfg, max_hits=ev.n)
    bufs = H.EventBuffers(plan, cap_peaks=256, cap_pairs=4096)
    x, y, lay, _ = H.hits_to_device(ev)
    bufs.run(H.make_hits(x, y, lay), cfg.threshold)
    torch.cuda.synchronize()
    _check(bufs.results(), gold)
    bb = H.BatchBuffers(plan, 3, 3 * ev.n, 256, 4096)
    bb.load([ev, ev, ev])
    bb.run(cfg.threshold)
    torch.cuda.synchronize()
    for e in range(3):
        _check(bb.results(e), gold)
