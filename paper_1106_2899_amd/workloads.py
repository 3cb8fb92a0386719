"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

The paper's runs are all synthetic equilibrium ensembles (Sec. 3.1 sampling
procedure) with the standard parameters of Sec. 4.1: N_0 = 4, N_s = 0.5,
zeta_s = 0.1, dt = 0.01.  These generators give the chain lengths, element
groupings and per-element velocity gradients of the benchmark workloads; the
same tables feed the GPU path and the oracle.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

STANDARD = dict(n0=4.0, ns=0.5, zeta_s=0.1, dt=0.01)


def shear(rate: float) -> np.ndarray:
    """Simple shear, kappa_xy = rate (Sec. 4.1 start-up shear)."""
    k = np.zeros((3, 3))
    k[0, 1] = rate
    return k


def uniaxial(rate: float) -> np.ndarray:
    """Uniaxial elongation, kappa = rate diag(1, -1/2, -1/2)."""
    return np.diag([rate, -0.5 * rate, -0.5 * rate])


def log_uniform(rng: np.random.Generator, lo: float, hi: float, size: int) -> np.ndarray:
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=size)


@dataclass
class Workload:
    name: str
    n_beads: np.ndarray                 # [M]
    element_offsets: np.ndarray         # [E+1]
    kappa: np.ndarray                   # [E][3][3]
    steps: int
    seed: int
    sample_every: int = 1
    rates: Optional[np.ndarray] = None  # [E] flow rate per element
    kinds: Optional[np.ndarray] = None  # [E] 0 shear, 1 uniaxial
    extra: dict = field(default_factory=dict)

    @property
    def n_chains(self) -> int:
        return int(self.n_beads.shape[0])

    @property
    def n_elements(self) -> int:
        return int(self.element_offsets.shape[0] - 1)

    @property
    def bead_steps(self) -> int:
        return int(self.n_beads.sum()) * self.steps


def _uniform_elements(M: int, E: int) -> np.ndarray:
    return (np.arange(E + 1, dtype=np.int64) * M // E).astype(np.int32)


def equilibrium_small(chains: int = 64, beads: int = 8, steps: int = 10_000, seed: int = 1) -> Workload:
    """64 chains of N = 8 at rest, 1e4 steps, sampled every step."""
    return Workload("equilibrium_64x8", np.full(chains, beads, np.int32), _uniform_elements(chains, 1),
                    np.zeros((1, 3, 3)), steps, seed, sample_every=1)


def linear_viscoelasticity(chains: int = 16384, beads: int = 32, steps: int = 100_000, seed: int = 2,
                           sample_every: int = 10) -> Workload:
    """16384 chains of N = 32 at rest for G(t) (multiple-tau correlator)."""
    return Workload("lve_16384x32", np.full(chains, beads, np.int32), _uniform_elements(chains, 1),
                    np.zeros((1, 3, 3)), steps, seed, sample_every=sample_every)


def startup_shear(elements: int = 4096, chains_per_element: int = 256, beads: int = 32, steps: int = 20_000,
                  seed: int = 3, sample_every: int = 10) -> Workload:
    """Fluid elements, each with its own shear rate log-uniform in [1e-4, 1]."""
    rng = np.random.default_rng(seed)
    rates = log_uniform(rng, 1e-4, 1.0, elements)
    M = elements * chains_per_element
    return Workload("startup_shear_4096x256x32", np.full(M, beads, np.int32), _uniform_elements(M, elements),
                    np.stack([shear(r) for r in rates]), steps, seed, sample_every=sample_every, rates=rates,
                    kinds=np.zeros(elements, np.int32))


def polydisperse(chains: int = 1 << 18, elements: int = 1024, steps: int = 10_000, seed: int = 4,
                 sample_every: int = 10) -> Workload:
    """N uniform in 16..128 per chain; per element shear or uniaxial
    elongation (probability 1/2 each) at a rate log-uniform in [1e-3, 0.1]."""
    rng = np.random.default_rng(seed)
    N = rng.integers(16, 129, size=chains).astype(np.int32)
    kinds = rng.integers(0, 2, size=elements).astype(np.int32)
    rates = log_uniform(rng, 1e-3, 0.1, elements)
    kap = np.stack([uniaxial(r) if t else shear(r) for t, r in zip(kinds, rates)])
    return Workload("polydisperse_2^18", N, _uniform_elements(chains, elements), kap, steps, seed,
                    sample_every=sample_every, rates=rates, kinds=kinds)


def differentiation(chains: int = 65536, beads: int = 64, steps: int = 2000, seed: int = 5,
                    rate: float = 0.01) -> Workload:
    """65536 chains of N = 64 under shear rate 0.01, 2000-step window."""
    return Workload("adjoint_65536x64", np.full(chains, beads, np.int32), _uniform_elements(chains, 1),
                    shear(rate)[None], steps, seed, sample_every=1, rates=np.array([rate]),
                    kinds=np.zeros(1, np.int32), extra={"checkpoint_every": 100})


def paper_table_shapes() -> list:
    """Table 1 shapes: N x M = 16x4096, 32x2048, 64x1024, 128x512, 1e4 steps."""
    return [(16, 4096), (32, 2048), (64, 1024), (128, 512)]
