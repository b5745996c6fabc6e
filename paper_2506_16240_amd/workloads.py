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
