"""Reader of the stored expected values under tests/golden/ (written by
tests/golden/make_golden.py from the CPU oracle)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_c1_event0():
    out = {"cands": [], "lists": []}
    with open(os.path.join(GOLDEN, "c1_event0.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, rest = line.split(None, 1)
            if key == "hits":
                n, _, digest = rest.split()
                out["hits"], out["digest"] = int(n), digest
            elif key in ("votes", "candidates", "pairs"):
                out[key] = int(rest)
            elif key == "cand":
                head, tail = rest.split(":")
                out["cands"].append([int(t) for t in head.split()])
                out["lists"].append([int(t) for t in tail.split()])
    out["cands"] = np.array(out["cands"], dtype=np.int32).reshape(-1, 4)
    return out


def read_cordic_table():
    rows = np.loadtxt(os.path.join(GOLDEN, "cordic_table.txt"), dtype=np.int64, comments="#")
    return rows[:, 1]
