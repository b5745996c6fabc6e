"""Serving pool: admission by HBM footprint, continuous batching, and results
that do not depend on the other jobs in the pool."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_16240_amd import micsa as M
from paper_2506_16240_amd import serve as SV


# ------------------------------------------------------------ CPU checks
def test_footprint_grows_with_size():
    a = M.footprint(8, 8, 8, 1, 1)
    b = M.footprint(16, 16, 16, 1, 1)
    c = M.footprint(16, 16, 16, 1, 4)
    assert 0 < a < b < c
    # byte layout: two state buffers of spin + daemon bytes, plus couplings
    assert b >= 4 * 16 ** 3


def test_submit_validation_without_device():
    pool = M.Pool(hbm_budget=1 << 20)
    sched = M.Schedule(M.SCHED_LINEAR, 3.0, 0.1, 100, 10)
    for bad in ((7, 8, 8), (8, 3, 8), (8, 8, 0)):
        with pytest.raises(M.MicsaError) as e:
            pool.submit(*bad, 1, 1, 1, sched)
        assert e.value.status == M.EINVAL
    with pytest.raises(M.MicsaError) as e:  # larger than the whole budget: could never run
        pool.submit(128, 128, 128, 1, 64, 1, sched)
    assert e.value.status == M.EINVAL
    with pytest.raises(M.MicsaError) as e:
        pool.submit(8, 8, 8, 1, 1, 1, M.Schedule(M.SCHED_CONST, -1.0, 1.0, 100, 10))
    assert e.value.status == M.EINVAL
    job = pool.submit(8, 8, 8, 1, 2, 1, sched)
    assert pool.state(job) == (M.JOB_QUEUED, 0)
    with pytest.raises(M.MicsaError):
        pool.release(job)  # not finished
    pool.close()


def test_job_stream_is_seeded():
    a = SV.job_stream(20, 50.0, 7)
    b = SV.job_stream(20, 50.0, 7)
    assert a == b
    assert all(s.L in SV.L_CHOICES and 1 <= s.R <= 64 for _, s in a)
    assert len({s.seed for _, s in a}) == 20
    assert all(t1 < t2 for (t1, _), (t2, _) in zip(a, a[1:]))


# ------------------------------------------------------------ GPU checks
def _run_alone(spec, sweeps_per_step):
    pool = M.Pool(1 << 34)
    job = pool.submit(spec.L, spec.L, spec.L, 1, spec.R, spec.seed,
                      M.Schedule(M.SCHED_LINEAR, spec.T0, spec.T1, spec.n_sweeps, spec.period))
    while pool.state(job)[0] != M.JOB_DONE:
        pool.step(sweeps_per_step)
    lat = pool.lattice(job)
    out = (lat.energy(), lat.spins(), lat.daemons(), lat.energy_tally())
    pool.release(job)
    pool.close()
    return out


TARGETS = [SV.JobSpec(16, 3, 0xC0FFEE, n_sweeps=300),   # batched resident launch
           SV.JobSpec(64, 2, 0xC0FFEF, n_sweeps=120),   # own stream, slab sweep
           SV.JobSpec(128, 1, 0xC0FFF0, n_sweeps=60),   # own stream, multispin planes
           SV.JobSpec(64, 20, 0xC0FFF1, n_sweeps=40)]   # own stream, bit planes (lanes = replicas)


def test_job_layout_policy():
    """L = 64 jobs of BITPLANE_MIN_REPLICAS or more replicas take the bit
    planes with lanes = replicas; every other job the byte layout."""
    for L in SV.L_CHOICES:
        for R in (1, SV.BITPLANE_MIN_REPLICAS - 1, SV.BITPLANE_MIN_REPLICAS, 64):
            layout, lanes = SV.job_layout(SV.JobSpec(L, R, 1))
            if L == 64 and R >= SV.BITPLANE_MIN_REPLICAS:
                assert (layout, lanes) == (M.LAYOUT_BITPLANE, M.LANES_REPLICAS)
            else:
                assert (layout, lanes) == (M.LAYOUT_BYTE, M.LANES_SAMPLES)


@pytest.mark.gpu
@pytest.mark.parametrize("target", TARGETS, ids=["L16-batched", "L64-slab", "L128-multispin", "L64-bitplane"])
def test_job_alone_equals_job_in_the_mix(target):
    """A job's final state is bit-identical alone (byte layout) and among
    other jobs that arrive before and after it, of other sizes, kernels and
    layouts, running concurrently on their own streams and in the batched
    launch, each in the layout the serving driver picks (the L = 64 target
    of 20 replicas in bit planes: layouts agree bit for bit); and it equals
    the oracle's trajectory."""
    alone = _run_alone(target, 37)
    others = [SV.JobSpec(8, 5, 11, n_sweeps=120), SV.JobSpec(32, 2, 12, n_sweeps=400),
              SV.JobSpec(64, 1, 13, n_sweeps=90), SV.JobSpec(16, 7, 14, n_sweeps=250),
              SV.JobSpec(128, 1, 15, n_sweeps=20), SV.JobSpec(64, 17, 16, n_sweeps=30)]
    pool = M.Pool(1 << 34)
    sub = lambda s: SV.submit(pool, s)
    ids = [sub(others[0]), sub(others[1])]
    pool.step(50)
    tid = sub(target)  # arrives while others are running
    ids.append(sub(others[2]))
    steps = 0
    while pool.state(tid)[0] != M.JOB_DONE:
        pool.step(37)
        steps += 1
        if steps == 2:
            ids += [sub(others[3]), sub(others[4]), sub(others[5])]
    lat = pool.lattice(tid)
    mixed = (lat.energy(), lat.spins(), lat.daemons())
    for a, b in zip(alone, mixed):
        assert np.array_equal(a, b)
    assert np.array_equal(alone[3], alone[0])  # the byte job's tally
    if SV.job_layout(target)[0] == M.LAYOUT_BYTE:
        assert np.array_equal(lat.energy_tally(), mixed[0])
    # (the bit-plane per-half sweep of L = 64 keeps no tally)
    # and the job equals the oracle's trajectory
    t = target
    o = O.Lattice(t.L, t.L, t.L, 1, t.R, t.seed)
    o.run(O.ALGO_MICSA, O.Schedule(O.SCHED_LINEAR, t.T0, t.T1, t.n_sweeps, t.period), t.n_sweeps, 0)
    assert np.array_equal(mixed[1], o.sigma) and np.array_equal(mixed[0], o.energy())
    assert np.array_equal(mixed[2], o.m)
    pool.sync()
    pool.close()


@pytest.mark.gpu
def test_admission_respects_the_budget():
    spec = SV.JobSpec(32, 4, 1, n_sweeps=60)
    fp = M.footprint(32, 32, 32, 1, 4)
    pool = M.Pool(int(fp * 2.5))  # room for two such jobs at a time
    jobs = [pool.submit(32, 32, 32, 1, 4, 100 + i, M.Schedule(M.SCHED_LINEAR, 3.0, 0.1, 60, 10)) for i in range(5)]
    seen = 0
    finished = set()
    t_end = time.monotonic() + 60
    while len(finished) < len(jobs) and time.monotonic() < t_end:
        running, queued = pool.step(20)  # enqueues without waiting for the device
        assert running <= 2
        seen = max(seen, running)
        for j in jobs:
            if j not in finished and pool.state(j)[0] == M.JOB_DONE:
                finished.add(j)
                pool.release(j)
        time.sleep(1e-3)
    assert seen == 2 and len(finished) == 5
    del spec
    pool.close()


@pytest.mark.gpu
def test_serve_short_stream():
    stream = SV.job_stream(12, 200.0, 3, n_sweeps=200)
    res, m = SV.serve(stream, hbm_budget=1 << 33, sweeps_per_step=50)
    assert m["jobs"] == 12 and all(np.isfinite(r.latency) and r.latency > 0 for r in res)
    assert m["p99_s"] >= m["p50_s"] > 0
    for r in res:
        N = r.spec.L ** 3
        assert len(r.energies) == r.spec.R and r.best_energy == r.energies.min()
        assert -3 * N <= r.best_energy <= 3 * N
