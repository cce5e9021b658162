"""Track-finding quality of a candidate list against the generator's truth (the efficiency and
purity of Sec. "Preliminary Results": fraction of simulated tracks reconstructed, and the
corresponding fraction of candidates that are real tracks).

The paper does not define a match.  Reading used here: a candidate is matched to generated track
t when at least `share` (default 75 %) of the hits on its list come from t; a generated track is
reconstructible when it left at least `min_hits` hits (default: the first-stage threshold), and
found when some candidate is matched to it.  Efficiency = found / reconstructible; purity =
matched candidates / candidates; duplicates = matched candidates per found track.

With background suppression inside the bin (hough_refine: one hit per layer from the densest
window of the angle inside the bin), the refined lists of the candidates that keep at least
`min_layers` layers are matched the same way (refined_csr builds their CSR lists).

A second reading, in parameter space (the figures show candidates as peaks at the generated
tracks' parameters): a generated track is found when a candidate lies within one bin of the bin
holding its true (d0, q/pT, phi0) in every direction (phi0 cyclic); purity = candidates within
one bin of some reconstructible track.  Host-side analysis of the outputs (numpy); nothing here
runs on the GPU.
"""
from __future__ import annotations

import numpy as np


def match_candidates(offsets: np.ndarray, hit_idx: np.ndarray, track_id: np.ndarray,
                     share: float = 0.75) -> np.ndarray:
    """Matched track of every candidate of a CSR list (-1: none).  offsets [n+1], hit_idx [pairs],
    track_id [hits] (-1 for noise)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    n = offsets.shape[0] - 1
    out = np.full(max(n, 0), -1, dtype=np.int64)
    if n <= 0 or offsets[-1] == 0:
        return out
    sizes = np.diff(offsets)
    cand = np.repeat(np.arange(n, dtype=np.int64), sizes)
    tid = np.asarray(track_id, dtype=np.int64)[np.asarray(hit_idx[: offsets[-1]], dtype=np.int64)]
    keep = tid >= 0
    cand, tid = cand[keep], tid[keep]
    if cand.size == 0:
        return out
    order = np.lexsort((tid, cand))
    cand, tid = cand[order], tid[order]
    new = np.ones(cand.size, dtype=bool)
    new[1:] = (cand[1:] != cand[:-1]) | (tid[1:] != tid[:-1])
    starts = np.flatnonzero(new)
    counts = np.diff(np.append(starts, cand.size))
    rc, rt = cand[starts], tid[starts]
    # the largest run per candidate (ties: the lower track id, which comes first)
    best = np.zeros(n, dtype=np.int64)
    best_t = np.full(n, -1, dtype=np.int64)
    order2 = np.lexsort((rt, -counts, rc))
    first = np.ones(order2.size, dtype=bool)
    first[1:] = rc[order2][1:] != rc[order2][:-1]
    sel = order2[first]
    best[rc[sel]] = counts[sel]
    best_t[rc[sel]] = rt[sel]
    ok = (sizes > 0) & (best >= share * sizes)
    out[ok] = best_t[ok]
    return out


def quality(offsets, hit_idx, track_id, n_tracks: int, min_hits: int, share: float = 0.75) -> dict:
    track_id = np.asarray(track_id)
    hits_per_track = np.bincount(track_id[track_id >= 0], minlength=n_tracks)[:n_tracks]
    recon = hits_per_track >= min_hits
    m = match_candidates(offsets, hit_idx, track_id, share)
    n_cand = m.shape[0]
    found = np.zeros(n_tracks, dtype=bool)
    found[m[m >= 0]] = True
    n_recon = int(recon.sum())
    n_found = int((found & recon).sum())
    n_matched = int((m >= 0).sum())
    return {
        "tracks": int(n_tracks), "reconstructible": n_recon, "found": n_found, "candidates": int(n_cand),
        "matched_candidates": n_matched,
        "efficiency": round(n_found / n_recon, 4) if n_recon else None,
        "purity": round(n_matched / n_cand, 4) if n_cand else None,
        "duplicates_per_found_track": round(n_matched / max(int(found.sum()), 1), 3),
    }


def true_bins(cfg, truth) -> np.ndarray:
    """Bin (l, k, b) holding each generated track's true parameters ([T][3]; l or k = -1 when
    outside the grid's range)."""
    phi = np.mod(np.asarray(truth["phi0"], dtype=np.float64), 2.0 * np.pi)
    b = np.minimum((phi / (2.0 * np.pi) * cfg.n_phi).astype(np.int64), cfg.n_phi - 1)
    qpt = np.asarray(truth["q"], dtype=np.float64) * np.asarray(truth["inv_pt"], dtype=np.float64)
    k = np.floor((qpt - cfg.qpt_min) / (cfg.qpt_max - cfg.qpt_min) * cfg.n_qpt).astype(np.int64)
    k = np.where((k >= 0) & (k < cfg.n_qpt), k, -1)
    if cfg.n_d0 == 1:
        l = np.zeros_like(k)
    else:
        d0 = np.asarray(truth["d0"], dtype=np.float64)
        l = np.floor((d0 - cfg.d0_min) / (cfg.d0_max - cfg.d0_min) * cfg.n_d0).astype(np.int64)
        l = np.where((l >= 0) & (l < cfg.n_d0), l, -1)
    if cfg.B_tesla == 0.0:
        k = np.zeros_like(k)  # no curvature: every q/pT row is the same line space; peaks sit in row 0
    return np.stack([l, k, b], axis=1)


def quality_params(cfg, truth, track_id, peaks: np.ndarray, min_hits: int) -> dict:
    """Parameter-space efficiency and purity of a candidate list (rows l, k, b, votes)."""
    track_id = np.asarray(track_id)
    n_tracks = len(truth["phi0"])
    hits_per_track = np.bincount(track_id[track_id >= 0], minlength=n_tracks)[:n_tracks]
    tb = true_bins(cfg, truth)
    recon = (hits_per_track >= min_hits) & (tb[:, 0] >= 0) & (tb[:, 1] >= 0)
    pk = np.asarray(peaks, dtype=np.int64).reshape(-1, 4)
    # candidate bins as keys; a track is found when any of the 27 neighbour keys holds a candidate
    def key(l, k, b):
        return (l * cfg.n_qpt + k) * cfg.n_phi + b
    cand = set(key(pk[:, 0], pk[:, 1], pk[:, 2]).tolist())
    found = np.zeros(n_tracks, dtype=bool)
    near = set()
    rb = tb[recon]
    ids = np.flatnonzero(recon)
    for dl in (-1, 0, 1):
        for dk in (-1, 0, 1):
            for db in (-1, 0, 1):
                l = rb[:, 0] + dl
                k = rb[:, 1] + dk
                b = np.mod(rb[:, 2] + db, cfg.n_phi)
                ok = (l >= 0) & (l < cfg.n_d0) & (k >= 0) & (k < cfg.n_qpt)
                keys = key(l, k, b)
                for t, kk, o in zip(ids, keys.tolist(), ok.tolist()):
                    if o:
                        near.add(kk)
                        if kk in cand:
                            found[t] = True
    n_recon = int(recon.sum())
    n_near = sum(1 for c in cand if c in near)
    return {"reconstructible": n_recon, "found": int(found.sum()), "candidates": len(cand),
            "candidates_near_a_track": n_near,
            "efficiency": round(int(found.sum()) / n_recon, 4) if n_recon else None,
            "purity": round(n_near / len(cand), 4) if cand else None}


def refined_csr(out_hits: np.ndarray, out_layers: np.ndarray, min_layers: int):
    """CSR lists of the refined candidates with at least `min_layers` layers: (offsets, hit_idx, kept
    candidate indices); each list holds its layers' hits in layer order."""
    out_hits = np.asarray(out_hits)
    keep = np.flatnonzero(np.asarray(out_layers) >= min_layers)
    rows = out_hits[keep]
    sizes = (rows >= 0).sum(axis=1)
    offsets = np.zeros(keep.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    return offsets, rows[rows >= 0].astype(np.int64), keep
