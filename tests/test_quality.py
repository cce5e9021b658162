"""Host-side quality analysis (efficiency and purity against the generator's truth) and the paper
detector's generator (straight lines, x/y smear).  CPU only."""
import math

import numpy as np

from paper_1305_4855_amd import configs, quality as Q, synth


def test_match_by_hit_share():
    # hits 0-9 track 0, 10-19 track 1, 20-29 track 2, 30-31 noise
    track_id = np.array([0] * 10 + [1] * 10 + [2] * 10 + [-1, -1], dtype=np.int32)
    lists = [list(range(10)),                      # track 0 exactly
             list(range(10, 15)) + list(range(20, 25)),  # half 1, half 2: no match
             list(range(20, 29)) + [30],           # 9 of 10 from track 2
             list(range(20, 26)) + [30, 31],       # 6 of 8 = 75 %: matched to 2 (duplicate)
             [],                                   # empty list
             [30, 31]]                             # noise only
    offs = np.concatenate([[0], np.cumsum([len(l) for l in lists])])
    idx = np.array([h for l in lists for h in l], dtype=np.int32)
    m = Q.match_candidates(offs, idx, track_id)
    assert m.tolist() == [0, -1, 2, 2, -1, -1]
    q = Q.quality(offs, idx, track_id, n_tracks=3, min_hits=8)
    assert q["reconstructible"] == 3 and q["found"] == 2 and q["candidates"] == 6
    assert q["efficiency"] == round(2 / 3, 4) and q["purity"] == 0.5
    assert q["duplicates_per_found_track"] == 1.5


def test_match_in_parameter_space():
    cfg = configs.C7.with_(n_tracks=3)
    truth = {"phi0": np.array([0.1, 3.0, 6.2]), "q": np.array([1.0, -1.0, 1.0]),
             "inv_pt": np.array([0.5, 0.25, 0.9]), "d0": np.zeros(3)}
    tb = Q.true_bins(cfg, truth)
    # phi0 bin and q/pT bin by their definitions
    assert tb[0].tolist() == [0, int((0.5 + 1.0) / 2.0 * 256), int(0.1 / (2 * math.pi) * 256)]
    track_id = np.repeat(np.arange(3), 10)
    pk = np.array([[0, tb[0, 1] + 1, tb[0, 2], 10],             # next to track 0
                   [0, tb[1, 1], (tb[1, 2] + 2) % 256, 10],     # two phi0 bins away from track 1
                   [0, tb[2, 1] - 1, (tb[2, 2] + 1) % 256, 10],  # diagonal neighbour of track 2 (phi0 wraps)
                   [0, 5, 5, 9]])                               # far from everything
    q = Q.quality_params(cfg, truth, track_id, pk, 8)
    assert q["found"] == 2 and q["candidates_near_a_track"] == 2 and q["efficiency"] == round(2 / 3, 4)
    assert q["purity"] == 0.5


def test_paper_detector_straight_lines():
    """50 straight lines, 10 hits each on layers at 11, 22, ..., 110 cm, smeared 0.4 mm in x and y:
    every hit lies near its line and its layer's radius."""
    cfg = configs.C6
    ev = synth.make_event(cfg, 1)
    assert ev.n == 500 and np.bincount(ev.layer).tolist() == [50] * 10
    t = ev.truth
    assert (np.abs(t["d0"]) <= 3.0).all()
    for k in range(50):
        sel = ev.track_id == k
        x, y = ev.x[sel].astype(np.float64), ev.y[sel].astype(np.float64)
        dist = -x * np.sin(t["phi0"][k]) + y * np.cos(t["phi0"][k]) - t["d0"][k]
        assert np.abs(dist).max() < 6 * 0.04 * math.sqrt(2)
        r = np.hypot(x, y)
        assert np.abs(r - np.asarray(cfg.radii_cm)[ev.layer[sel]]).max() < 6 * 0.04 * math.sqrt(2)
        # outgoing: hits lie ahead of the PCA along the direction phi0
        assert ((x * np.cos(t["phi0"][k]) + y * np.sin(t["phi0"][k])) > 0).all()
