"""Host-side logic that needs no GPU: the benchmark's single-GPU contract and its algorithmic-byte
formulas, the autotuner's cache keys and kernel-path rule, and the XCD placement of a batch's
events (the snake over the size order must give every event to exactly one XCD)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bench_byte_formulas():
    sys.path.insert(0, ROOT)
    import bench

    # the dense event's figures: 236 899 candidates, 7 001 027 pairs, 32 MiB accumulator
    assert bench.assign_hbm_bytes(236899, 7001027) == 20 * 236899 + 4 + 4 * 7001027
    acc = 512 * 256 * 64 * 4
    assert bench.chain_hbm_bytes(acc, 236899, 7001027, 1) == 2 * acc + 36 * 236899 + 4 + 4 * 7001027
    # a batch counts one closing CSR offset per event
    assert bench.chain_hbm_bytes(acc, 10, 20, 3) - bench.chain_hbm_bytes(acc, 10, 20, 1) == 8


def test_tuner_keys_and_paths():
    from paper_1305_4855_amd import configs, tune

    c2, c4, c1 = configs.C2, configs.C4, configs.C1
    assert tune.path_of(c2, 16384) == "pt" and tune.path_of(c2, 65536) == "slab"
    assert tune.path_of(c1.with_(n_phi=64), 100) == "slab"
    k_single = tune.cache_key(c2, "gfx950", 16384, "single")
    k_batch = tune.cache_key(configs.C3, "gfx950", configs.C3.max_hits_per_event, "batch")
    assert k_single == "gfx950:512x256x64:i32:f7:pt:single" and k_batch == "gfx950:512x256x64:i32:f7:pt:batch"
    assert tune.cache_key(c4, "gfx950", 32767, "batch") == "gfx950:1024x512x128:i16:f7:pt:batch"
    assert tune.cache_key(c2.with_(frac_bits=8), "gfx950", 16384, "single") != k_single
    # every cached entry names only known knobs, with values from the search space or the defaults
    cache = json.load(open(tune.CACHE))
    for key, entry in cache.items():
        mode = key.rsplit(":", 1)[1]
        assert set(entry["best"]) == set(tune.DEFAULT), key
        for knob, v in entry["best"].items():
            assert v == tune.DEFAULT[knob] or v in tune.SPACE[mode].get(knob, ()), (key, knob, v)


def _xcd_rank(g, x, xcds=8):
    """The placement rule of the batched vote and assignment, restated: XCD x takes size rank
    8g + x for even g and 8g + 7 - x for odd g."""
    return xcds * g + ((xcds - 1 - x) if g & 1 else x)


@pytest.mark.parametrize("n_events", [1, 2, 7, 8, 9, 64, 255, 256])
def test_xcd_placement_covers_every_event_once(n_events):
    groups = (n_events + 7) // 8
    seen = [(x, _xcd_rank(g, x)) for x in range(8) for g in range(groups) if _xcd_rank(g, x) < n_events]
    ranks = sorted(r for _, r in seen)
    assert ranks == list(range(n_events))
    # the snake balances: over whole groups every XCD's ranks sum to the same total
    if n_events % 8 == 0 and groups % 2 == 0:
        sums = {x: sum(r for xx, r in seen if xx == x) for x in range(8)}
        assert len(set(sums.values())) == 1


def test_xcd_rank_matches_the_kernel_source():
    src = open(os.path.join(ROOT, "paper_1305_4855_amd", "csrc", "hough.hip")).read()
    assert "kXcds * g + ((g & 1) ? kXcds - 1 - x : x)" in src
