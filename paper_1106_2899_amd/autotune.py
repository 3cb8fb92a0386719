"""Autotuner for the chain-to-wavefront mapping of the step kernel.

Chains are bucketed by length into the classes (2..8], (8..16], (16..32],
(32..64], (64..128].  For every class present in an ensemble the tuner times
each supported mapping (W lanes per chain, B beads per lane, W*B >= the
longest chain of the class) on a probe ensemble made of a sample of that
class's chains, sampled at the ensemble's own stress interval, using the
library's kernel timing mode (HIP events around the step-kernel launches),
and applies the fastest mapping.  Given the ensemble's velocity-gradient
table, every probe chain runs under its own element's kappa, so that the
timing includes the flow terms the workload executes.  Trajectories do not
depend on the mapping, so tuning never changes results.
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
    """ns per bead-step of `mapping` on chains of `lengths`; kappa: None (at
    rest) or [len(lengths)][9], one element per chain."""
    import torch

    from .ensemble import Ensemble

    lo, hi = int(lengths.min()), int(lengths.max())
    M = len(lengths)
    E = 1 if kappa is None else M
    e = Ensemble(lengths, n_elements=E, element_offsets=None if kappa is None else np.arange(M + 1),
                 precision=precision, seed=seed, corr_levels=0, use_graph=False, sample_every=sample_every,
                 max_steps_per_launch=steps, device=device)
    try:
        k = None if kappa is None else torch.as_tensor(np.ascontiguousarray(kappa, dtype=np.float64).reshape(M, 9),
                                                       device=e.device)
        e.set_mapping(lo, hi, mapping[0], mapping[1])
        e.init()
        e.step(steps, k)  # warm-up launch
        e.set_kernel_timing(True)
        e.step(steps, k)
        e.step(steps, k)
        ms, launches, bead_steps = e.kernel_time()
        return ms * 1e6 / bead_steps
    finally:
        e.close()


def tune(ensemble, kappa=None, *, steps: int = 200, probe_chains: int = 16384, seed: int = 12345,
         cache: Optional[str] = None, apply: bool = True) -> TuneResult:
    """Times every candidate mapping per length class of `ensemble` and applies
    the fastest.  kappa: the ensemble's velocity gradients [E][9] (or [E][3][3];
    None: at rest), so that probes run the workload's flow terms.  `cache`:
    optional JSON file of previous choices (keyed by precision, class and
    whether there is flow) that is reused when present."""
    res = TuneResult()
    cached = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            cached = json.load(f)
    kap_chain = None
    if kappa is not None:
        k = np.asarray(kappa.detach().cpu() if hasattr(kappa, "detach") else kappa, dtype=np.float64)
        k = k.reshape(-1, 9)
        if k.shape[0] == 1:
            k = np.repeat(k, ensemble.n_elements, axis=0)
        if np.any(k != 0.0):
            kap_chain = np.repeat(k, np.diff(np.asarray(ensemble.element_offsets, dtype=np.int64)), axis=0)
    key_prefix = ensemble.precision + (":flow" if kap_chain is not None else "")
    N = ensemble.N
    rng = np.random.default_rng(seed)
    for lo, hi in CLASSES:
        idx = np.nonzero((N >= lo) & (N <= hi))[0]
        if idx.size == 0:
            continue
        sel = N[idx]
        ckey = f"{key_prefix}:{lo}-{hi}"
        if ckey in cached:
            best = tuple(cached[ckey])
        else:
            pick = np.sort(rng.choice(idx, size=probe_chains, replace=False)) if idx.size > probe_chains else idx
            probe = np.ascontiguousarray(N[pick], dtype=np.int32)
            pk = None if kap_chain is None else kap_chain[pick]
            times = {}
            for m in candidates(int(sel.max())):
                times[m] = _time_mapping(probe, m, ensemble.precision, steps, seed, pk, ensemble.device,
                                         ensemble.sample_every)
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
