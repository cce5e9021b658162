"""Seeded synthetic events shaped like the paper's standalone Monte Carlo.

The paper's simulation (Sec. "Preliminary Results") is a transverse-plane
detector model of concentric layers with Gaussian hit smearing; its curved
tracks come from the interaction point and its new triggers look for tracks
from displaced vertices (Sec. "New Trigger Capabilities").  This module draws
such events for the workloads in ``configs``: helical tracks through a barrel
of cylindrical layers in a solenoidal field, one hit at the first crossing of
each layer, r-phi smearing, uniformly distributed noise hits, displaced tracks
and long-lived-particle decay vertices.

It contains none of the Hough transform's arithmetic: hit positions come from
circle-circle intersection geometry, not from the transform's
phi0 = phi - asin(A) relation.  Both the GPU path and the CPU oracle take the
float32 hits produced here as their input.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .configs import HoughConfig, get

SEED_BASE = 13054855
C_LIGHT = 0.299792458  # GeV / (T m)


@dataclasses.dataclass
class Event:
    x: np.ndarray            # float32 [n]
    y: np.ndarray            # float32 [n]
    z: Optional[np.ndarray]  # float32 [n] or None
    layer: np.ndarray        # uint8 [n]
    track_id: np.ndarray     # int32 [n], -1 for noise
    truth: dict              # per-track arrays: q, inv_pt, phi0, d0, z0, cot, kind, vertex
                             # (-1 or the index of the track's decay vertex); vertices [n][2]

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _rng(cfg: HoughConfig, event_id: int) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, cfg.cfg_id, event_id])


def _radius_cm(inv_pt: np.ndarray, B: float) -> np.ndarray:
    # bending radius R[m] = pT / (0.2998 B) ; in cm
    return 100.0 / (C_LIGHT * B * inv_pt)


def _first_crossings(cx, cy, R, sense, px, py, radii):
    """First crossing of each layer circle |X| = r by the circle of centre (cx, cy)
    and radius R, travelled from the point (px, py) in rotation sense
    `sense` (+1 counter-clockwise, -1 clockwise), within half a turn.

    Arrays of shape [T] for the circle, [L] for radii.  Returns
    (x, y, arc, ok) of shape [T, L]."""
    cx = cx[:, None]; cy = cy[:, None]; R = R[:, None]; sense = sense[:, None]
    r = np.asarray(radii, dtype=np.float64)[None, :]
    dC = np.hypot(cx, cy)
    dC_safe = np.where(dC > 0, dC, 1.0)
    a = (r * r - R * R + dC * dC) / (2.0 * dC_safe)
    h2 = r * r - a * a
    ok = (h2 >= 0.0) & (dC > 0)
    h = np.sqrt(np.where(ok, h2, 0.0))
    ux, uy = cx / dC_safe, cy / dC_safe
    vx, vy = -uy, ux
    psi0 = np.arctan2(py[:, None] - cy, px[:, None] - cx)
    best_x = np.zeros(np.broadcast(cx, r).shape)
    best_y = np.zeros_like(best_x)
    best_d = np.full_like(best_x, np.inf)
    for sgn in (1.0, -1.0):
        X = a * ux + sgn * h * vx
        Y = a * uy + sgn * h * vy
        psi = np.arctan2(Y - cy, X - cx)
        d = np.mod(sense * (psi - psi0), 2.0 * np.pi)
        take = d < best_d
        best_x = np.where(take, X, best_x)
        best_y = np.where(take, Y, best_y)
        best_d = np.where(take, d, best_d)
    ok = ok & (best_d <= np.pi)
    return best_x, best_y, best_d * R, ok


def _smear_rphi(rng, x, y, sigma):
    r = np.hypot(x, y)
    phi = np.arctan2(y, x) + rng.normal(0.0, sigma, size=x.shape) / np.where(r > 0, r, 1.0)
    return r * np.cos(phi), r * np.sin(phi)


def _n_tracks(cfg: HoughConfig, rng) -> int:
    if cfg.track_dist == "fixed":
        return int(cfg.n_tracks)
    if cfg.track_dist == "gamma_poisson":
        # mean ~ track_mean, long tail; clipped to the stated range
        lam = rng.gamma(2.0, cfg.track_mean / 2.0)
        n = int(rng.poisson(lam))
        lo, hi = cfg.track_range
        return int(min(max(n, lo), hi))
    raise ValueError(cfg.track_dist)


def _helix_hits(rng, cfg, q, inv_pt, phi0, d0, z0, cot, start=None, r_min=None):
    """Hits of tracks given by perigee parameters.  If `start` (vx, vy, s_offset)
    is given, tracks are followed from that point (decay vertex) and only layers
    with radius > r_min are crossed."""
    B = cfg.B_tesla
    if B == 0.0:
        return _line_hits(rng, cfg, phi0, d0)
    R = _radius_cm(inv_pt, B)
    nx, ny = -np.sin(phi0), np.cos(phi0)
    px, py = d0 * nx, d0 * ny
    # positive charges turn clockwise for B along +z: centre on the right of the motion
    cx, cy = px - q * R * nx, py - q * R * ny
    sense = -q
    if start is not None:
        sx, sy = start
    else:
        sx, sy = px, py
    X, Y, arc, ok = _first_crossings(cx, cy, R, sense, sx, sy, cfg.radii_cm)
    if r_min is not None:
        ok &= np.asarray(cfg.radii_cm)[None, :] > r_min[:, None]
    T, L = X.shape
    X, Y = _smear_rphi(rng, X, Y, cfg.smear_rphi_cm)
    if cfg.smear_xy_cm > 0.0:
        X = X + rng.normal(0.0, cfg.smear_xy_cm, size=X.shape)
        Y = Y + rng.normal(0.0, cfg.smear_xy_cm, size=Y.shape)
    Z = None
    if cfg.with_z:
        if start is not None:
            # arc measured from the vertex; the vertex z is z0 + s_vertex * cot
            s_pca_to_start = _arc_from_pca(cx, cy, R, sense, px, py, sx, sy)
            Z = z0[:, None] + (s_pca_to_start[:, None] + arc) * cot[:, None]
        else:
            Z = z0[:, None] + arc * cot[:, None]
        Z = Z + rng.normal(0.0, cfg.smear_z_cm, size=Z.shape)
        ok &= np.abs(Z) <= np.asarray(cfg.halflen_cm)[None, :]
    lay = np.broadcast_to(np.arange(L, dtype=np.uint8)[None, :], (T, L))
    tid = np.broadcast_to(np.arange(T, dtype=np.int32)[:, None], (T, L))
    return X[ok], Y[ok], (Z[ok] if Z is not None else None), lay[ok], tid[ok]


def _line_hits(rng, cfg, phi0, d0):
    """Hits of straight lines (no field): the line through the PCA d0 * (-sin phi0, cos phi0) with
    direction phi0 meets each layer it reaches once on its way out; smeared in x and y."""
    r = np.asarray(cfg.radii_cm, dtype=np.float64)[None, :]
    d = d0[:, None]
    ok = r > np.abs(d)
    t = np.sqrt(np.where(ok, r * r - d * d, 0.0))
    X = -d * np.sin(phi0)[:, None] + t * np.cos(phi0)[:, None]
    Y = d * np.cos(phi0)[:, None] + t * np.sin(phi0)[:, None]
    if cfg.smear_xy_cm > 0.0:
        X = X + rng.normal(0.0, cfg.smear_xy_cm, size=X.shape)
        Y = Y + rng.normal(0.0, cfg.smear_xy_cm, size=Y.shape)
    T, L = X.shape
    lay = np.broadcast_to(np.arange(L, dtype=np.uint8)[None, :], (T, L))
    tid = np.broadcast_to(np.arange(T, dtype=np.int32)[:, None], (T, L))
    Z = None
    if cfg.with_z:
        Z = np.zeros_like(X)
    return X[ok], Y[ok], (Z[ok] if Z is not None else None), lay[ok], tid[ok]


def _arc_from_pca(cx, cy, R, sense, px, py, sx, sy):
    psi0 = np.arctan2(py - cy, px - cx)
    psi1 = np.arctan2(sy - cy, sx - cx)
    return R * np.mod(sense * (psi1 - psi0), 2.0 * np.pi)


def _perigee_from_vertex(vx, vy, alpha, q, inv_pt, B):
    """Perigee (phi0, d0) of the circle through (vx, vy) with direction alpha."""
    R = _radius_cm(inv_pt, B)
    nx, ny = -np.sin(alpha), np.cos(alpha)
    cx, cy = vx - q * R * nx, vy - q * R * ny
    dC = np.hypot(cx, cy)
    # closest point of the circle to the origin
    px, py = cx - R * cx / dC, cy - R * cy / dC
    sense = -q
    # tangent of the motion at the PCA
    tx, ty = -sense * (py - cy) / R, sense * (px - cx) / R
    phi0 = np.mod(np.arctan2(ty, tx), 2.0 * np.pi)
    d0 = px * (-np.sin(phi0)) + py * np.cos(phi0)
    return phi0, d0


def make_event(cfg, event_id: int = 0) -> Event:
    cfg = get(cfg)
    rng = _rng(cfg, event_id)
    nt = _n_tracks(cfg, rng)
    q = rng.choice(np.array([-1.0, 1.0]), size=nt)
    inv_pt = rng.uniform(0.01, 1.0, size=nt)
    phi0 = rng.uniform(0.0, 2.0 * np.pi, size=nt)
    d0 = np.zeros(nt)
    disp = rng.random(nt) < cfg.displaced_frac
    nd = int(disp.sum())
    d0[disp] = rng.choice(np.array([-1.0, 1.0]), size=nd) * rng.uniform(0.0, cfg.displaced_d0_max, size=nd)
    eta = rng.uniform(-1.0, 1.0, size=nt)
    cot = np.sinh(eta)
    z0 = rng.normal(0.0, 5.0, size=nt)
    xs, ys, zs, ls, ts = _helix_hits(rng, cfg, q, inv_pt, phi0, d0, z0, cot)
    kinds = [np.zeros(nt, dtype=np.int8)]
    truth_q, truth_ipt, truth_phi0, truth_d0, truth_z0, truth_cot = [q], [inv_pt], [phi0], [d0], [z0], [cot]
    parts = [(xs, ys, zs, ls, ts)]
    n_tracks_total = nt
    vert_of = [np.full(nt, -1, dtype=np.int32)]
    vertices = []
    if cfg.n_llp_vertices > 0:
        zpv = rng.normal(0.0, 5.0)
        for _ in range(cfg.n_llp_vertices):
            rv = rng.uniform(*cfg.llp_r_range)
            phiv = rng.uniform(0.0, 2.0 * np.pi)
            cotv = np.sinh(rng.uniform(-1.0, 1.0))
            zv = zpv + rv * cotv
            lo, hi = cfg.llp_daughters
            nd_ = int(rng.integers(lo, hi + 1))
            vx, vy = rv * np.cos(phiv), rv * np.sin(phiv)
            vert_of.append(np.full(nd_, len(vertices), dtype=np.int32))
            vertices.append((vx, vy))
            dq, dipt, dalpha, dphi0, dd0 = [], [], [], [], []
            while len(dq) < nd_:
                qq = float(rng.choice(np.array([-1.0, 1.0])))
                ipt = float(rng.uniform(0.01, 1.0))
                alpha = phiv + float(rng.uniform(-0.5, 0.5))
                p0, dd = _perigee_from_vertex(np.array([vx]), np.array([vy]), np.array([alpha]),
                                              np.array([qq]), np.array([ipt]), cfg.B_tesla)
                if abs(dd[0]) > cfg.llp_d0_max:
                    continue
                dq.append(qq); dipt.append(ipt); dalpha.append(alpha); dphi0.append(p0[0]); dd0.append(dd[0])
            dq, dipt, dphi0, dd0 = map(np.asarray, (dq, dipt, dphi0, dd0))
            dcot = cotv + rng.normal(0.0, 0.3, size=nd_)
            # z at the PCA such that the helix passes through the vertex
            R = _radius_cm(dipt, cfg.B_tesla)
            nx, ny = -np.sin(dphi0), np.cos(dphi0)
            px, py = dd0 * nx, dd0 * ny
            cx, cy = px - dq * R * nx, py - dq * R * ny
            s_v = _arc_from_pca(cx, cy, R, -dq, px, py, np.full(nd_, vx), np.full(nd_, vy))
            dz0 = zv - s_v * dcot
            xs, ys, zs, ls, ts = _helix_hits(rng, cfg, dq, dipt, dphi0, dd0, dz0, dcot,
                                             start=(np.full(nd_, vx), np.full(nd_, vy)),
                                             r_min=np.full(nd_, rv))
            parts.append((xs, ys, zs, ls, ts + n_tracks_total))
            n_tracks_total += nd_
            truth_q.append(dq); truth_ipt.append(dipt); truth_phi0.append(dphi0); truth_d0.append(dd0)
            truth_z0.append(dz0); truth_cot.append(dcot); kinds.append(np.ones(nd_, dtype=np.int8))
    x = np.concatenate([p[0] for p in parts])
    y = np.concatenate([p[1] for p in parts])
    z = np.concatenate([p[2] for p in parts]) if cfg.with_z else None
    lay = np.concatenate([p[3] for p in parts]).astype(np.uint8)
    tid = np.concatenate([p[4] for p in parts]).astype(np.int32)
    n_track_hits = x.shape[0]
    n_noise = int(round(cfg.noise_frac * n_track_hits))
    if n_noise:
        radii = np.asarray(cfg.radii_cm)
        nl = rng.choice(len(radii), size=n_noise, p=radii / radii.sum())
        nphi = rng.uniform(0.0, 2.0 * np.pi, size=n_noise)
        x = np.concatenate([x, radii[nl] * np.cos(nphi)])
        y = np.concatenate([y, radii[nl] * np.sin(nphi)])
        if z is not None:
            hl = np.asarray(cfg.halflen_cm)[nl]
            z = np.concatenate([z, rng.uniform(-1.0, 1.0, size=n_noise) * hl])
        lay = np.concatenate([lay, nl.astype(np.uint8)])
        tid = np.concatenate([tid, np.full(n_noise, -1, dtype=np.int32)])
    perm = rng.permutation(x.shape[0])
    truth = dict(q=np.concatenate(truth_q), inv_pt=np.concatenate(truth_ipt),
                 phi0=np.concatenate(truth_phi0), d0=np.concatenate(truth_d0),
                 z0=np.concatenate(truth_z0), cot=np.concatenate(truth_cot),
                 kind=np.concatenate(kinds), vertex=np.concatenate(vert_of),
                 vertices=np.asarray(vertices, dtype=np.float64).reshape(-1, 2))
    return Event(
        x=np.ascontiguousarray(x[perm], dtype=np.float32),
        y=np.ascontiguousarray(y[perm], dtype=np.float32),
        z=(np.ascontiguousarray(z[perm], dtype=np.float32) if z is not None else None),
        layer=np.ascontiguousarray(lay[perm], dtype=np.uint8),
        track_id=np.ascontiguousarray(tid[perm], dtype=np.int32),
        truth=truth)


def make_events(cfg, n: Optional[int] = None, first: int = 0):
    cfg = get(cfg)
    n = cfg.n_events if n is None else n
    return [make_event(cfg, first + i) for i in range(n)]


def pack_events(events):
    """CSR packing of several events: concatenated SoA hits + offsets[n_events+1]."""
    offs = np.zeros(len(events) + 1, dtype=np.int32)
    offs[1:] = np.cumsum([e.n for e in events])
    x = np.concatenate([e.x for e in events]) if events else np.zeros(0, np.float32)
    y = np.concatenate([e.y for e in events]) if events else np.zeros(0, np.float32)
    lay = np.concatenate([e.layer for e in events]) if events else np.zeros(0, np.uint8)
    z = None
    if events and events[0].z is not None:
        z = np.concatenate([e.z for e in events])
    return x, y, z, lay, offs


def make_candidates(cfg, n: int, seed: int = 0, votes=(7, 12)) -> np.ndarray:
    """A synthetic candidate list of the first transform's shape: n distinct bins (l, k, b)
    of the config's grid in increasing linear index, each with a vote count drawn uniformly
    from [votes[0], votes[1]].  Rows (l, k, b, votes), int32.  Input of the second transform
    at full size without running the first one."""
    cfg = get(cfg)
    rng = np.random.default_rng([13054855, cfg.cfg_id, 1 << 20, seed])
    nb = cfg.n_bins
    n = int(min(n, nb))
    lin = np.sort(rng.choice(nb, size=n, replace=False)) if n else np.zeros(0, np.int64)
    out = np.empty((n, 4), dtype=np.int32)
    out[:, 0] = lin // (cfg.n_qpt * cfg.n_phi)
    out[:, 1] = (lin // cfg.n_phi) % cfg.n_qpt
    out[:, 2] = lin % cfg.n_phi
    out[:, 3] = rng.integers(votes[0], votes[1] + 1, size=n)
    return out
