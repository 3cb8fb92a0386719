"""Autotuner for the chain-to-wavefront mapping of the step kernel.

Chains are bucketed by length into the classes (2..8], (8..16], (16..32],
(32..64], (64..128].  For every class present in an ensemble the tuner times
each supported mapping (W lanes per chain, B beads per lane, W*B >= the
longest chain of the class) on a probe ensemble made of a sample of that
class's chains, sampled at the ensemble's own stress interval, using the
library's kernel timing mode (HIP events around the step-kernel launches),
and applies the fastest mapping.  Trajectories do not depend on the mapping,
so tuning never changes results.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

CLASSES = [(2, 8), (9, 16), (17, 32), (33, 64), (65, 128)]
MAPPINGS = [(8, 1), (16, 1), (32, 1), (64, 1), (16, 2), (32, 2), (64, 2)]


def candidates(n_max: int) -> List[Tuple[int, int]]:
    return [(w, b) for (w, b) in MAPPINGS if w * b >= n_max]


@dataclass
class TuneResult:
    choices: Dict[Tuple[int, int], Tuple[int, int]] = field(default_factory=dict)
    timings: Dict[Tuple[int, int], Dict[Tuple[int, int], float]] = field(default_factory=dict)  # ns per bead-step

    def to_json(self) -> str:
        return json.dumps({
            "choices": {f"{lo}-{hi}": list(m) for (lo, hi), m in self.choices.items()},
            "timings_ns_per_bead_step": {f"{lo}-{hi}": {f"{w}x{b}": t for (w, b), t in d.items()}
                                         for (lo, hi), d in self.timings.items()},
        })


def _time_mapping(lengths: np.ndarray, mapping, precision: str, steps: int, seed: int, kappa, device,
                  sample_every: int = 1) -> float:
    from .ensemble import Ensemble

    lo, hi = int(lengths.min()), int(lengths.max())
    e = Ensemble(lengths, precision=precision, seed=seed, corr_levels=0, use_graph=False, sample_every=sample_every,
                 max_steps_per_launch=steps, device=device)
    try:
        e.set_mapping(lo, hi, mapping[0], mapping[1])
        e.init()
        e.step(steps, kappa)  # warm-up launch
        e.set_kernel_timing(True)
        e.step(steps, kappa)
        e.step(steps, kappa)
        ms, launches, bead_steps = e.kernel_time()
        return ms * 1e6 / bead_steps
    finally:
        e.close()


def tune(ensemble, *, steps: int = 200, probe_chains: int = 16384, seed: int = 12345,
         cache: Optional[str] = None, apply: bool = True) -> TuneResult:
    """Times every candidate mapping per length class of `ensemble` and applies
    the fastest.  `cache`: optional JSON file of previous choices (keyed by
    precision and class) that is reused when present."""
    res = TuneResult()
    cached = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            cached = json.load(f)
    key_prefix = ensemble.precision
    N = ensemble.N
    rng = np.random.default_rng(seed)
    for lo, hi in CLASSES:
        sel = N[(N >= lo) & (N <= hi)]
        if sel.size == 0:
            continue
        ckey = f"{key_prefix}:{lo}-{hi}"
        if ckey in cached:
            best = tuple(cached[ckey])
        else:
            probe = rng.choice(sel, size=min(probe_chains, sel.size), replace=False) if sel.size > probe_chains else sel
            times = {}
            for m in candidates(int(sel.max())):
                times[m] = _time_mapping(np.ascontiguousarray(probe, dtype=np.int32), m, ensemble.precision, steps,
                                         seed, None, ensemble.device, ensemble.sample_every)
            res.timings[(lo, hi)] = times
            best = min(times, key=times.get)
            cached[ckey] = list(best)
        res.choices[(lo, hi)] = best
        if apply:
            ensemble.set_mapping(int(sel.min()), int(sel.max()), best[0], best[1])
    if cache:
        with open(cache, "w") as f:
            json.dump(cached, f, indent=1)
    return res
