"""Write the stored expected values under tests/golden/ from the CPU oracle.

Every value here is computed by oracle/ (and the seeded input generator);
nothing comes from the GPU library.  Run from the repository root:

    python tests/golden/make_golden.py

c1_event0.txt   the small single-event workload (10 prompt tracks, 256 phi0 x 256
                q/pT bins, threshold 8), event 0: a digest of its hits, the vote
                total, every candidate (l, k, b, votes) and its hit list.
cordic_table.txt  the 30 CORDIC angles T_i = round(atan(2^-i) * 2^31 / pi) of the
                azimuth (Volder's vectoring rotations), from a 50-digit evaluation,
                next to the oracle's own table read back through or_azimuth.
"""
import hashlib
import os
import sys

import mpmath as mp
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1305_4855_amd import configs, synth  # noqa: E402


def hits_digest(ev) -> str:
    h = hashlib.sha256()
    for a in (ev.x, ev.y, ev.layer):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:32]


def write_c1(path: str) -> None:
    cfg = configs.C1
    ev = synth.make_event(cfg, 0)
    g = O.Cfg(cfg)
    acc, nv = O.vote(g, ev)
    n, pk = O.peaks(g, acc, cfg.threshold)
    offs, hit_idx, tot = O.assign(g, ev, pk)
    with open(path, "w") as f:
        f.write("# c1 event 0: 10 prompt tracks, 256x256x1 int32, threshold 8 (written by make_golden.py)\n")
        f.write(f"hits {ev.n} digest {hits_digest(ev)}\n")
        f.write(f"votes {nv}\n")
        f.write(f"candidates {n}\n")
        f.write(f"pairs {tot}\n")
        for i in range(n):
            l, k, b, v = (int(t) for t in pk[i])
            hs = " ".join(str(int(h)) for h in hit_idx[offs[i]:offs[i + 1]])
            f.write(f"cand {l} {k} {b} {v} : {hs}\n")


def write_cordic(path: str) -> None:
    mp.mp.dps = 50
    with open(path, "w") as f:
        f.write("# i  T_i = round(atan(2^-i) * 2^31 / pi), 50-digit evaluation (written by make_golden.py)\n")
        for i in range(30):
            t = mp.atan(mp.mpf(2) ** (-i)) * mp.mpf(2) ** 31 / mp.pi
            f.write(f"{i} {int(mp.nint(t))}\n")


if __name__ == "__main__":
    write_c1(os.path.join(HERE, "c1_event0.txt"))
    write_cordic(os.path.join(HERE, "cordic_table.txt"))
    print("written")
