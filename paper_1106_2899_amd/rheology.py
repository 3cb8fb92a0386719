"""Start-up shear, steady viscosity and the Cox-Merz comparison (Sec. 4.1).

For t > 0 the ensemble is sheared with kappa_xy = gdot from equilibrium; the
viscosity growth is eta(t, gdot) = <sigma_xy(t)> / gdot and the steady
viscosity eta(gdot) its long-time limit.  The Cox-Merz rule compares
eta(gdot) with the dynamic viscosity |eta*(w)| = |G'(w) + i G''(w)| / w at
w = gdot.  Also reported: the mean number of slip-springs <Z> in the steady
state.

Everything runs on the device through the library (the element series gives
sum_k sigma_xy,k per sample); this module only schedules the runs and
averages their outputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from .ensemble import Ensemble


@dataclass
class StartupShear:
    rate: float
    t: np.ndarray          # sample times
    eta_plus: np.ndarray   # eta(t, gdot) per sample
    eta: float             # steady viscosity: mean of eta_plus over the tail window
    eta_err: float         # batch-means error of that mean (8 blocks)
    z_mean: float          # <Z> at the end of the run
    z_eq: float            # <Z> at the start (equilibrium)


def mean_springs(e: Ensemble) -> float:
    """<Z>: occupied slots per chain in the current state."""
    _, _, S = e.state()
    return float((S >= 0).sum().item()) / e.M


def startup_shear(n_beads: int, n_chains: int, rate: float, steps: int, *, sample_every: int = 10,
                  tail: float = 0.5, precision: str = "fp32", seed: int = 3, construct_rule: int = 0,
                  device: Optional[str] = None) -> StartupShear:
    """Shear an equilibrium ensemble at kappa_xy = rate for `steps` steps;
    eta(gdot) averages eta(t, gdot) over the last `tail` fraction of the run."""
    if rate <= 0.0:
        raise ValueError("rate must be positive")
    q = steps // sample_every
    e = Ensemble(n_beads, n_chains, precision=precision, seed=seed, sample_every=sample_every, corr_levels=0,
                 series_capacity=q, construct_rule=construct_rule, device=device)
    try:
        e.init()
        z_eq = mean_springs(e)
        kap = np.zeros((3, 3))
        kap[0, 1] = rate
        e.step(steps, kap)
        ser = e.element_series().cpu().numpy()  # [E][T][6]
        sxy = ser[0, :q, 3] / n_chains      # <sigma_xy>(t)
        t = (np.arange(q) + 1) * sample_every * e.dt
        eta_plus = sxy / rate
        n_tail = max(8, int(tail * q))
        tw = eta_plus[q - n_tail:]
        blocks = np.array([b.mean() for b in np.array_split(tw, 8)])
        z_mean = mean_springs(e)
    finally:
        e.close()
    return StartupShear(rate=rate, t=t, eta_plus=eta_plus, eta=float(tw.mean()),
                        eta_err=float(blocks.std(ddof=1) / math.sqrt(len(blocks))), z_mean=z_mean, z_eq=z_eq)


def cox_merz(steady: Sequence[StartupShear], eta_abs_at_rates: Sequence[float]) -> Dict[str, np.ndarray]:
    """eta(gdot) beside |eta*(w = gdot)| and their ratio."""
    rates = np.array([s.rate for s in steady])
    eta = np.array([s.eta for s in steady])
    star = np.asarray(eta_abs_at_rates, dtype=np.float64)
    return {"rate": rates, "eta": eta, "eta_star": star, "ratio": eta / star}
