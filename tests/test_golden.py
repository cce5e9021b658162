"""The oracle against the stored expected values in tests/golden/ (a
regression pin for the small single-event workload) and the CORDIC angle table
against its 50-digit evaluation."""
import hashlib
import math

import numpy as np

from paper_1305_4855_amd import configs, synth
from tests.golden_io import read_c1_event0, read_cordic_table


def test_c1_event0_reproduced_by_oracle(oracle_mod):
    O = oracle_mod
    gold = read_c1_event0()
    cfg = configs.C1
    ev = synth.make_event(cfg, 0)
    h = hashlib.sha256()
    for a in (ev.x, ev.y, ev.layer):
        h.update(np.ascontiguousarray(a).tobytes())
    assert ev.n == gold["hits"] and h.hexdigest()[:32] == gold["digest"]
    g = O.Cfg(cfg)
    acc, nv = O.vote(g, ev)
    assert nv == gold["votes"] == ev.n * cfg.n_qpt  # every prompt sample of this grid is valid
    n, pk = O.peaks(g, acc, cfg.threshold)
    assert n == gold["candidates"]
    np.testing.assert_array_equal(pk, gold["cands"])
    offs, hit_idx, tot = O.assign(g, ev, pk)
    assert tot == gold["pairs"]
    for i, lst in enumerate(gold["lists"]):
        assert list(hit_idx[offs[i]:offs[i + 1]]) == lst
    # every generated track peaks: its ten hits form one candidate list
    tracks = {}
    for hit, t in enumerate(ev.track_id):
        tracks.setdefault(int(t), set()).add(hit)
    lists = [set(l) for l in gold["lists"]]
    for t, hits in tracks.items():
        if t >= 0:
            assert any(hits <= l for l in lists), t


def test_cordic_table_50_digits_equals_double_rounding():
    table = read_cordic_table()
    assert len(table) == 30
    for i, t in enumerate(table):
        assert t == round(math.atan(2.0 ** -i) * (2147483648.0 / math.pi)), i
    assert list(table[:4]) == [536870912, 316933406, 167458907, 85004756]
