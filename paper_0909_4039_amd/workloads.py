"""Named synthetic workloads (sizes and physical parameters only; no arithmetic).

They follow the paper's problem statement (Sec. 2: an m-mode of the s = -2
Teukolsky equation on an (r*, theta) grid, a particle source on a circular
equatorial orbit, a waveform read at an extraction radius).  The paper
prints no grid sizes; these are synthetic stand-ins.  Where a workload does
not fix the r* range it uses [-100, 400].
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict
from typing import Optional

import numpy as np


@dataclass
class Workload:
    name: str
    nr: int
    nth: int
    rstar_min: float
    rstar_max: float
    a: float
    m: int
    s: int = -2
    M: float = 1.0
    steps: int = 1000
    r0: float = 0.0          # source orbit radius (0: no source)
    amp: float = 0.0
    rstar_obs: float = 100.0
    pulse: Optional[dict] = None   # {"center":, "width":, "seed":}
    extra: dict = field(default_factory=dict)

    def as_dict(self):
        return asdict(self)


SCHWARZSCHILD_PULSE = Workload(
    "schwarzschild_pulse_256x64", nr=256, nth=64, rstar_min=-50.0, rstar_max=150.0,
    a=0.0, m=2, steps=2000, rstar_obs=100.0, pulse={"center": 20.0, "width": 4.0, "seed": 1})

KERR_SOURCE = Workload(
    "kerr_a0.9_source_8192x256", nr=8192, nth=256, rstar_min=-100.0, rstar_max=400.0,
    a=0.9, m=2, steps=50000, r0=10.0, amp=1.0, rstar_obs=300.0)

# At the stable dt, 20000 steps cover T = 21.6 M; signals from the source
# (r* = 12.8) and the pulse (r* = 20) reach r* = 30 within the run but need
# ~280 M to reach r* = 300, so gradient checks read the misfit at r* = 30.
ADJOINT = Workload(
    "adjoint_a0.6_4096x256", nr=4096, nth=256, rstar_min=-100.0, rstar_max=400.0,
    a=0.6, m=2, steps=20000, r0=10.0, amp=1.0, rstar_obs=300.0,
    pulse={"center": 20.0, "width": 4.0, "seed": 4}, extra={"rstar_obs_reached": 30.0})

LARGE = Workload(
    "kerr_a0.99_source_32768x1024", nr=32768, nth=1024, rstar_min=-100.0, rstar_max=400.0,
    a=0.99, m=2, steps=100000, r0=8.0, amp=1.0, rstar_obs=100.0)


def batched_instances(seed: int = 3):
    """32 instances: m = 1..8 x a in {0, 0.3, 0.6, 0.9}; uneven grids drawn from default_rng(seed).

    N_r* ~ U{2048..16384}, N_theta ~ U{64..512}; pulse centre U[0, 50], width U[2, 6],
    amplitude 1 + 0.1 (2U - 1); source r0 ~ U[6, 12], amp = 1.
    """
    rng = np.random.default_rng(seed)
    out = []
    for m in range(1, 9):
        for a in (0.0, 0.3, 0.6, 0.9):
            nr = int(rng.integers(2048, 16385))
            nth = int(rng.integers(64, 513))
            c = float(rng.uniform(0.0, 50.0))
            w = float(rng.uniform(2.0, 6.0))
            A = float(1.0 + 0.1 * (2.0 * rng.random() - 1.0))
            r0 = float(rng.uniform(6.0, 12.0))
            out.append(Workload(f"batch_m{m}_a{a}", nr=nr, nth=nth, rstar_min=-100.0,
                                rstar_max=400.0, a=a, m=m, steps=10000, r0=r0, amp=1.0,
                                rstar_obs=100.0,
                                pulse={"center": c, "width": w, "amplitude": A}))
    return out


def adjoint_perturbation(seed: int = 4):
    """Relative perturbations (eps_r0, eps_amp, eps_pulse) ~ U[-0.02, 0.02] for the target run."""
    rng = np.random.default_rng(seed)
    e = rng.uniform(-0.02, 0.02, size=3)
    return float(e[0]), float(e[1]), float(e[2])
