"""Synthetic workloads: lattice sizes, seeds and schedules of the five
configurations this library is measured and tested on.

This module only describes inputs; every number the method computes comes
from the HIP library (or, in tests, from the CPU oracle).  Inputs follow the
paper's distributions: couplings +-1 with probability 1/2 (Sec. 2.1), an
infinite-temperature random start (Sec. 3) and daemons drawn from eq.
prob-daemons-walkers -- all generated from the seed by the counter-based
generator, identically on both sides.  The paper's own sample (one L = 160
lattice, Sec. 3) is not available; these seeded samples stand in for it.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SCHED_CONST, SCHED_LINEAR = 0, 1


@dataclass(frozen=True)
class Workload:
    name: str
    Lx: int
    Ly: int
    Lz: int
    S: int           # samples
    R: int           # replicas per sample
    seed: int
    kind: int        # temperature schedule kind
    T0: float
    T1: float
    n_sweeps: int
    period: int      # daemon refresh period
    layout: int = 0  # 0 byte, 1 bit-plane

    @property
    def N(self) -> int:
        return self.Lx * self.Ly * self.Lz

    @property
    def lattices(self) -> int:
        return self.S * self.R

    def updates(self, sweeps: int | None = None) -> int:
        """Spin updates = sites x lattices x sweeps (every visited site counts)."""
        return self.N * self.lattices * (self.n_sweeps if sweeps is None else sweeps)


PARAMAGNET_L16 = Workload("paramagnet_L16", 16, 16, 16, 1, 1, 0x5EED0001, SCHED_CONST, 1.5, 1.5, 1000, 10)
QUENCH_L64 = Workload("quench_L64_T0.7", 64, 64, 64, 1, 2, 0x5EED0002, SCHED_CONST, 0.7, 0.7, 100000, 10)
BATCHED_L32 = Workload("batched_L32_256x2", 32, 32, 32, 256, 2, 0x5EED0003, SCHED_CONST, 0.8, 0.8, 10000, 10)
ANNEAL_L512 = Workload("anneal_L512_T3.0-0.2", 512, 512, 512, 1, 1, 0x5EED0004, SCHED_LINEAR, 3.0, 0.2, 10000,
                       20)

ALL = {w.name: w for w in (PARAMAGNET_L16, QUENCH_L64, BATCHED_L32, ANNEAL_L512)}


# ----------------------------------------------------------- App. C workload
def gaussian_couplings(Lx: int, Ly: int, Lz: int, seed: int) -> np.ndarray:
    """One sample of Gaussian couplings J ~ N(0, 1) (App. C) as [3, N]: row mu
    holds the bond (i, i + e_mu), site i = x + Lx (y + Ly z).  Values beyond
    |J| = 8 (probability about 1e-15 per bond) are clipped to the range the
    library accepts."""
    rng = np.random.default_rng(seed)
    return np.clip(rng.standard_normal((3, Lx * Ly * Lz)), -8.0, 8.0)


@dataclass(frozen=True)
class PTWorkload:
    """Parallel tempering of one Gaussian sample: runs independent runs, each
    with 2 replicas of M clones at temperatures uniform in [Tmin, Tmax]; an
    EMCS is `sweeps` sweeps per clone, a Houdayer move per temperature and a
    tempering step per replica (App. C)."""
    name: str
    L: int
    runs: int
    M: int
    Tmin: float
    Tmax: float
    sweeps: int
    seed: int

    @property
    def N(self) -> int:
        return self.L ** 3

    def temperatures(self) -> np.ndarray:
        return np.linspace(self.Tmin, self.Tmax, self.M)

    def couplings(self) -> np.ndarray:
        return gaussian_couplings(self.L, self.L, self.L, self.seed)

    def updates(self, emcs: int) -> int:
        """Spin updates: every site of every clone once per sweep."""
        return self.N * 2 * self.M * self.runs * self.sweeps * emcs


# the paper's App. C set-up (L = 10, N_R = 2, N_beta = 40, T in [0.2, 2], 10
# sweeps per EMCS) with 200 independent runs of the sample, as in its Table 4
PT_L10 = PTWorkload("pt_gauss_L10_200x2x40", 10, 200, 40, 0.2, 2.0, 10, 0x5EED0006)
