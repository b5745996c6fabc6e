"""Annealing service driver: Poisson arrivals into a continuous-batching pool.

Jobs are instances of the 3D EA +-J model with L uniform in {8, 16, 32, 64,
128} and 1..64 replicas of one sample, annealed with MicSA from T = 3.0 to
0.1 over 2000 sweeps (refresh every 10 sweeps), each in the layout
job_layout() picks for its size.  Arrivals follow a Poisson
process of the given rate; each arrival is submitted to the pool as soon as
its time has passed.  The loop calls the pool's step over and over: each
call admits what fits and enqueues the next `sweeps_per_step` sweeps of
every job whose previous chunks have finished, without waiting for the
device, so jobs run concurrently (each large job on its own stream, the
small ones in one batched launch) while new arrivals are admitted.  The time to solution of a job is its completion time minus its arrival
time.  All device work happens in libmicsa.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import micsa as M

L_CHOICES = (8, 16, 32, 64, 128)
# L = 64 jobs with at least this many replicas run in the bit-plane layout
BITPLANE_MIN_REPLICAS = 16


def splitmix64(x: int) -> int:
    """Job seed from (stream seed, job id): the SplitMix64 finaliser."""
    x = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return x ^ (x >> 31)


@dataclass
class JobSpec:
    L: int
    R: int
    seed: int
    T0: float = 3.0
    T1: float = 0.1
    n_sweeps: int = 2000
    period: int = 10

    @property
    def updates(self) -> int:
        return self.L ** 3 * self.R * self.n_sweeps


@dataclass
class JobResult:
    spec: JobSpec
    arrival: float
    done: float = float("nan")
    best_energy: int = 0
    energies: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def job_layout(spec: "JobSpec") -> tuple[int, int]:
    """(layout, lane mode) a job runs in.  L = 64 jobs of many replicas take
    the bit-plane layout with lanes = replicas: a word holds one site of up
    to 64 replicas of the instance, the couplings broadcast to every lane
    (multispin coding of replicas, Sec. 2.5).  There it beats the byte
    slab sweep from about 16 replicas on (1.2x at 20, 1.8x at 37, 2.4x at
    53 on one MI355X), and loses below.  Every other job keeps the byte
    layout: the batched resident launch for L <= 32, the multispin planes
    for L = 128 (faster than bit planes at every replica count there).
    Results do not depend on the layout."""
    if spec.L == 64 and spec.R >= BITPLANE_MIN_REPLICAS:
        return M.LAYOUT_BITPLANE, M.LANES_REPLICAS
    return M.LAYOUT_BYTE, M.LANES_SAMPLES


def submit(pool: "M.Pool", spec: "JobSpec") -> int:
    """Submit a job in the layout job_layout() picks."""
    layout, lanes = job_layout(spec)
    return pool.submit(spec.L, spec.L, spec.L, 1, spec.R, spec.seed,
                       M.Schedule(M.SCHED_LINEAR, spec.T0, spec.T1, spec.n_sweeps, spec.period),
                       layout=layout, lane_mode=lanes)


def job_stream(n_jobs: int, rate: float, seed: int, n_sweeps: int = 2000, L_choices=L_CHOICES,
               max_replicas: int = 64) -> list[tuple[float, JobSpec]]:
    """Poisson arrivals (exponential gaps of mean 1/rate seconds) with random sizes."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for j in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        spec = JobSpec(int(rng.choice(L_choices)), int(rng.integers(1, max_replicas + 1)),
                       splitmix64((seed << 20) ^ j), n_sweeps=n_sweeps)
        out.append((t, spec))
    return out


def serve(stream: list[tuple[float, JobSpec]], hbm_budget: int, sweeps_per_step: int = 100,
          max_running: int = 1 << 20, poll_s: float = 2e-4) -> tuple[list[JobResult], dict]:
    """Run the arrival stream through a pool; returns per-job results and metrics."""
    pool = M.Pool(hbm_budget, max_running)
    results: dict[int, JobResult] = {}
    pending = list(stream)
    t0 = time.perf_counter()
    live: set[int] = set()
    max_running_seen = 0
    while pending or live:
        now = time.perf_counter() - t0
        while pending and pending[0][0] <= now:
            arr, spec = pending.pop(0)
            job = submit(pool, spec)
            results[job] = JobResult(spec, arr)
            live.add(job)
        if not live:
            time.sleep(max(0.0, min(pending[0][0] - now, 0.05)))
            continue
        # enqueue the next chunk of every job with a free slot; the call does
        # not wait for the device, so arrivals keep being admitted while it runs
        running, _ = pool.step(sweeps_per_step)
        max_running_seen = max(max_running_seen, running)
        now = time.perf_counter() - t0
        finished = 0
        for job in list(live):
            st, _ = pool.state(job)
            if st == M.JOB_DONE:
                lat = pool.lattice(job)
                E = lat.energy()
                r = results[job]
                r.done, r.energies, r.best_energy = now, E, int(E.min())
                pool.release(job)
                live.discard(job)
                finished += 1
        if not finished:
            time.sleep(poll_s)  # every job has work in flight: poll again shortly
    wall = time.perf_counter() - t0
    pool.close()
    res = [results[j] for j in sorted(results)]
    lat = np.array([r.latency for r in res])
    upd = sum(r.spec.updates for r in res)
    metrics = {"jobs": len(res), "wall_s": wall, "p50_s": float(np.percentile(lat, 50)),
               "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
               "updates_per_ns": upd / (wall * 1e9), "max_running": max_running_seen}
    return res, metrics


def capacity(specs: list[JobSpec], hbm_budget: int, sweeps_per_step: int) -> float:
    """Service capacity in spin updates/ns: these jobs, all arriving at once."""
    _, m = serve([(0.0, spec) for spec in specs], hbm_budget, sweeps_per_step)
    return m["updates_per_ns"]


def main() -> int:
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Poisson job stream through the continuous-batching pool: "
                                             "p50/p99 time to solution, throughput, best energy per job.")
    ap.add_argument("--jobs", type=int, default=60)
    ap.add_argument("--loads", default="0.5,0.8,1.0", help="offered loads as fractions of the measured capacity")
    ap.add_argument("--seed", type=int, default=0x5EED0005)
    ap.add_argument("--sweeps", type=int, default=2000)
    ap.add_argument("--sweeps-per-step", type=int, default=100)
    ap.add_argument("--hbm-gib", type=float, default=64.0)
    ap.add_argument("--capacity-runs", type=int, default=3, help="capacity is the median of this many runs")
    args = ap.parse_args()
    budget = int(args.hbm_gib * (1 << 30))
    # the job sizes do not depend on the arrival rate (the gaps scale one
    # exponential draw each), so every load level serves this same mix
    specs = [spec for _, spec in job_stream(args.jobs, 1.0, args.seed, args.sweeps)]
    runs = [capacity(specs, budget, args.sweeps_per_step) for _ in range(max(1, args.capacity_runs))]
    cap = float(np.median(runs))
    mean_updates = float(np.mean([s.updates for s in specs]))
    print(json.dumps({"capacity_updates_per_ns": round(cap, 1), "capacity_runs": [round(r, 1) for r in runs],
                      "mean_job_updates": mean_updates}), flush=True)
    for load in (float(x) for x in args.loads.split(",")):
        rate = load * cap * 1e9 / mean_updates  # jobs per second
        res, m = serve(job_stream(args.jobs, rate, args.seed, args.sweeps), budget, args.sweeps_per_step)
        e_best = [r.best_energy / r.spec.L ** 3 for r in res]
        print(json.dumps({"load": load, "rate_jobs_per_s": round(rate, 3), **{k: (round(v, 4) if isinstance(v, float)
                          else v) for k, v in m.items()}, "best_e_per_spin_mean": round(float(np.mean(e_best)), 4),
                          "best_e_per_spin_min": round(float(np.min(e_best)), 4)}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
