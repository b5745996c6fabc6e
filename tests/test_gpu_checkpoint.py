"""Checkpoint and resume through the C ABI (micsa_save / micsa_load).

A run split at any sweep k -- save, a fresh context created from the same
parameters, load, continue -- must equal the continuous run bit for bit:
every random number depends on (seed, sample, replica, site, sweep or
refresh index) only, so the saved state plus k is the whole state.  The
cases cover the byte layout on the fused sweep, the multispin sweep with a
walker wandering still owed at the split, the bit-plane layout, six walker
families, the heat bath, and the oracle's own trajectory.
"""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_16240_amd import micsa as M

pytestmark = pytest.mark.gpu


def _state(g):
    out = {"spins": g.spins(), "daemons": g.daemons(), "E": g.energy(), "D": g.daemon_energy(),
           "k": g.counters()[0]}
    try:
        out["tally"] = g.energy_tally()
    except M.MicsaError:
        out["tally"] = None
    return out


def _assert_same(a, b):
    for key in a:
        if a[key] is None:
            assert b[key] is None
        else:
            assert np.array_equal(a[key], b[key]), key


CASES = [
    # (id, shape, layout, gamma, algo, kernel, schedule (kind, T0, T1, n, P), split)
    ("byte_fused", (128, 16, 8, 1, 2), M.LAYOUT_BYTE, 1, M.ALGO_MICSA, M.KERNEL_FUSED,
     (M.SCHED_LINEAR, 2.5, 0.5, 30, 4), 13),
    ("multispin_walkers_owed", (256, 16, 8, 1, 1), M.LAYOUT_BYTE, 1, M.ALGO_WALKERS, M.KERNEL_MULTISPIN,
     (M.SCHED_LINEAR, 2.0, 0.6, 30, 5), 13),
    ("multispin_daemons", (256, 16, 8, 1, 1), M.LAYOUT_BYTE, 1, M.ALGO_MICSA, M.KERNEL_MULTISPIN,
     (M.SCHED_LINEAR, 2.0, 0.6, 30, 5), 9),
    ("bitplane", (32, 8, 8, 70, 2), M.LAYOUT_BITPLANE, 1, M.ALGO_MICSA, M.KERNEL_AUTO,
     (M.SCHED_CONST, 0.8, 0.8, 30, 10), 11),
    ("gamma6_walkers", (16, 8, 8, 1, 2), M.LAYOUT_BYTE, 6, M.ALGO_WALKERS, M.KERNEL_AUTO,
     (M.SCHED_CONST, 1.2, 1.2, 30, 2), 7),
    ("heatbath_table", (32, 8, 6, 2, 1), M.LAYOUT_BYTE, 1, M.ALGO_HEATBATH, M.KERNEL_AUTO,
     (M.SCHED_TABLE, 0, 0, 30, 10), 16),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_split_run_equals_continuous_run(case):
    _, shape, layout, gamma, algo, kernel, (kind, T0, T1, n, P), split = case
    table = np.array([2.0, 1.1, 0.7]) if kind == M.SCHED_TABLE else None
    sched = M.Schedule(kind, T0, T1, n, P, table)
    seed = 0xC0FFEE

    def make():
        g = M.Lattice(*shape, seed, layout=layout, gamma=gamma)
        g.set_option(M.OPT_SWEEP_KERNEL, kernel)
        return g

    a = make()
    a.set_schedule(sched)
    a.sweep(algo, n)
    want = _state(a)
    a.close()

    b = make()
    b.set_schedule(sched)
    b.sweep(algo, split)
    image = b.save()
    b.sweep(algo, 3)  # work after the save must not leak into the image
    b.close()
    c = make()  # no schedule: the image brings it
    c.load(image)
    assert c.counters()[0] == split
    c.sweep(algo, n - split)
    _assert_same(want, _state(c))
    # rewinding a used context to the image continues identically too
    c.load(image)
    c.sweep(algo, n - split)
    _assert_same(want, _state(c))
    c.close()


def test_split_run_equals_oracle():
    """The resumed byte-layout run against the oracle's continuous trajectory."""
    shape, seed, n, split = (64, 8, 8, 2, 2), 77, 24, 10
    gs = M.Schedule(M.SCHED_LINEAR, 3.0, 0.4, n, 6)
    os_ = O.Schedule(O.SCHED_LINEAR, 3.0, 0.4, n, 6)
    o = O.Lattice(*shape, seed)
    o.run(O.ALGO_MICSA, os_, n, 0)
    g = M.Lattice(*shape, seed)
    g.set_schedule(gs)
    g.sweep(M.ALGO_MICSA, split)
    image = g.save()
    g.close()
    h = M.Lattice(*shape, seed)
    h.load(image)
    h.sweep(M.ALGO_MICSA, n - split)
    assert np.array_equal(h.spins(), o.sigma) and np.array_equal(h.daemons(), o.m)
    assert np.array_equal(h.energy(), o.energy()) and np.array_equal(h.energy_tally(), o.energy())
    h.close()


def test_load_rejects_foreign_or_damaged_images():
    g = M.Lattice(32, 8, 8, 1, 2, 5)
    g.set_schedule(M.Schedule(M.SCHED_CONST, 1.0, 1.0, 20, 5))
    g.sweep(M.ALGO_MICSA, 4)
    image = g.save()
    before = _state(g)
    # too small a buffer: ERANGE and the size
    n = ctypes.c_size_t(len(image) - 1)
    buf = ctypes.create_string_buffer(len(image))
    assert M.lib().micsa_save(g._ctx, buf, ctypes.byref(n)) == M.ERANGE and n.value == len(image)
    damaged = bytearray(image)
    damaged[len(image) // 2] ^= 1
    for bad in (bytes(damaged), image[:-1], b"x" * len(image)):
        assert M.lib().micsa_load(g._ctx, bad, len(bad)) == M.EINVAL
    for other in (M.Lattice(32, 8, 8, 1, 2, 6), M.Lattice(32, 8, 8, 1, 1, 5), M.Lattice(32, 8, 10, 1, 2, 5)):
        assert M.lib().micsa_load(other._ctx, image, len(image)) == M.EINVAL
        other.close()
    _assert_same(before, _state(g))  # nothing changed by the refused loads
    g.close()
