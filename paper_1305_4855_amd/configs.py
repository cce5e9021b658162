"""Workload definitions: detector geometry, parameter grid and event generator
settings of the five synthetic workloads.

Plain data only (no arithmetic of the transform).  The detector is a barrel of
ten cylindrical layers with CMS-like radii (the paper's inner-tracker section
describes the CMS barrel; its own toy detector is ten evenly spaced layers);
the field is 3.8 T.  Grid ranges cover the generated 1/pT in [0.01, 1] GeV^-1
and |d0| up to 10 cm (20 cm for the long-lived-particle search).
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

RADII_CM: Tuple[float, ...] = (4.4, 7.3, 10.2, 25.5, 33.9, 41.8, 49.8, 60.8, 69.2, 78.0)
# half-lengths grow linearly from 30 cm (innermost) to 110 cm (outermost)
HALFLEN_CM: Tuple[float, ...] = tuple(30.0 + 80.0 * i / 9.0 for i in range(10))
B_TESLA = 3.8


@dataclasses.dataclass(frozen=True)
class HoughConfig:
    name: str
    cfg_id: int
    # detector
    radii_cm: Tuple[float, ...] = RADII_CM
    halflen_cm: Tuple[float, ...] = HALFLEN_CM
    B_tesla: float = B_TESLA
    # parameter grid: phi0 x q/pT x d0, accumulator acc[l][k][b] (b = phi0 bin fastest)
    n_phi: int = 512
    n_qpt: int = 256
    n_d0: int = 64
    frac_bits: int = 7          # angle bits below one phi0 bin
    qpt_min: float = -1.0
    qpt_max: float = 1.0
    d0_min: float = -10.0
    d0_max: float = 10.0
    acc_bits: int = 32
    threshold: int = 7
    # second-stage r-z vote (cot(theta) x z0), only for the LLP search
    n_cot: int = 0
    n_z0: int = 0
    cot_min: float = -2.0
    cot_max: float = 2.0
    z0_min: float = -32.0
    z0_max: float = 32.0
    # second transform over the candidates (displaced-jet vertices): n_vr radius rows over
    # [vr_min, vr_max) cm times n_vphi azimuth bins (0 = none); candidates with fewer than
    # v_min_votes votes (0 = the first-stage threshold, i.e. all) do not vote
    n_vr: int = 0
    n_vphi: int = 0
    vr_min: float = 0.0
    vr_max: float = 32.0
    v_min_votes: int = 0
    v_threshold: int = 3
    # event generator
    n_events: int = 1
    n_tracks: int = 1000            # fixed count (when track_dist == "fixed")
    track_dist: str = "fixed"       # "fixed" | "gamma_poisson"
    track_mean: float = 500.0
    track_range: Tuple[int, int] = (50, 2000)
    noise_frac: float = 0.2
    displaced_frac: float = 0.1
    displaced_d0_max: float = 10.0
    smear_rphi_cm: float = 20e-4
    smear_xy_cm: float = 0.0        # Gaussian smear of x and y each (the paper's own detector model)
    smear_z_cm: float = 50e-4
    with_z: bool = False
    n_llp_vertices: int = 0
    llp_r_range: Tuple[float, float] = (1.0, 30.0)
    llp_daughters: Tuple[int, int] = (2, 6)
    llp_d0_max: float = 20.0
    # serving
    rate_hz: float = 0.0
    duration_s: float = 0.0
    hbm_budget_bytes: int = 0
    max_hits_per_event: int = 32767

    @property
    def n_layers(self) -> int:
        return len(self.radii_cm)

    @property
    def n_bins(self) -> int:
        return self.n_phi * self.n_qpt * self.n_d0

    @property
    def acc_bytes(self) -> int:
        return self.n_bins * self.acc_bits // 8

    def with_(self, **kw) -> "HoughConfig":
        return dataclasses.replace(self, **kw)


C1 = HoughConfig(
    name="c1_single_event_2d", cfg_id=1, n_phi=256, n_qpt=256, n_d0=1, d0_min=0.0, d0_max=0.0,
    threshold=8, n_tracks=10, noise_frac=0.0, displaced_frac=0.0)

C2 = HoughConfig(
    name="c2_dense_event_3d", cfg_id=2, n_phi=512, n_qpt=256, n_d0=64, threshold=7,
    n_tracks=1000, noise_frac=0.2, displaced_frac=0.1)

C3 = HoughConfig(
    name="c3_batched_uneven", cfg_id=3, n_phi=512, n_qpt=256, n_d0=64, threshold=7,
    n_events=256, track_dist="gamma_poisson", track_mean=500.0, noise_frac=0.2,
    displaced_frac=0.05)

C4 = HoughConfig(
    name="c4_llp_search", cfg_id=4, n_phi=1024, n_qpt=512, n_d0=128, frac_bits=7,
    d0_min=-20.0, d0_max=20.0, acc_bits=16, threshold=7, n_cot=128, n_z0=128,
    n_events=64, n_tracks=600, noise_frac=0.2, displaced_frac=0.0, with_z=True,
    n_llp_vertices=2, n_vr=64, n_vphi=512)

C5 = HoughConfig(
    name="c5_streaming_trigger", cfg_id=5, n_phi=512, n_qpt=256, n_d0=64, threshold=7,
    track_dist="gamma_poisson", track_mean=500.0, noise_frac=0.2, displaced_frac=0.05,
    rate_hz=20000.0, duration_s=60.0, hbm_budget_bytes=64 << 30)

# The paper's own detector model (Sec. "Preliminary Results", detector paragraph): a 3.0 cm beam pipe
# and ten concentric, evenly spaced layers, the last at 110.0 cm (read as 11, 22, ..., 110 cm), hit
# resolution 0.4 mm in x and in y.
PAPER_RADII_CM: Tuple[float, ...] = tuple(11.0 * (i + 1) for i in range(10))

# Fig. "hough": 50 straight-line tracks with 10 hits each (B = 0; lines with |d0| up to the beam pipe
# radius).  Straight lines have no curvature, so every q/pT row of the grid is the same line space.
C6 = HoughConfig(
    name="c6_paper_straight_lines", cfg_id=6, radii_cm=PAPER_RADII_CM, halflen_cm=(110.0,) * 10, B_tesla=0.0,
    n_phi=256, n_qpt=64, n_d0=64, d0_min=-4.0, d0_max=4.0, threshold=8, n_tracks=50, noise_frac=0.0,
    displaced_frac=1.0, displaced_d0_max=3.0, smear_rphi_cm=0.0, smear_xy_cm=0.04)

# The curved-track example (Sec. "Preliminary Results", curved-track paragraph): prompt tracks, the
# two-parameter phi0 x q/pT space, on the paper's detector; track count varied for the efficiency
# and purity against the number of tracks.
C7 = HoughConfig(
    name="c7_paper_curved_prompt", cfg_id=7, radii_cm=PAPER_RADII_CM, halflen_cm=(110.0,) * 10, B_tesla=B_TESLA,
    n_phi=256, n_qpt=256, n_d0=1, d0_min=0.0, d0_max=0.0, threshold=8, n_tracks=1000, noise_frac=0.0,
    displaced_frac=0.0, smear_rphi_cm=0.0, smear_xy_cm=0.04)

CONFIGS = {c.cfg_id: c for c in (C1, C2, C3, C4, C5, C6, C7)}


def get(cfg: "int | str | HoughConfig") -> HoughConfig:
    if isinstance(cfg, HoughConfig):
        return cfg
    if isinstance(cfg, int):
        return CONFIGS[cfg]
    s = str(cfg).lower()
    for c in CONFIGS.values():
        if s == c.name or s == f"c{c.cfg_id}":
            return c
    raise KeyError(cfg)


def small_variant(base: HoughConfig, n_tracks: int = 40, n_phi: Optional[int] = None,
                  n_qpt: Optional[int] = None, n_d0: Optional[int] = None) -> HoughConfig:
    """A reduced grid/event of the same shape family, for parity tests the oracle
    finishes in seconds (several slabs and a ragged hit tail)."""
    return base.with_(
        name=base.name + "_small", n_tracks=n_tracks, track_dist="fixed", n_events=1,
        n_phi=n_phi or base.n_phi, n_qpt=n_qpt or base.n_qpt, n_d0=n_d0 or base.n_d0)
