"""GPU: the device-pointer logging call and full-length state hashes.

micsa_sweep_logged_d writes the energy and daemon logs into device arrays in
stream order; its rows must equal those of micsa_sweep_logged (host arrays)
and the oracle's, on every sweep path: the resident kernel, the per-half
kernels, the slab, the fused byte sweep, the multispin and bit-plane
layouts, and the heat bath.

The configurations' full schedules are too long for the oracle beyond
their first sweeps, so they are checked by state hashes at k = 10^j: on the
512^3 anneal the multispin sweep (the bench's path), the fused byte sweep
and the per-half kernels; on the 64^3 quench (10^5 sweeps) the two-sweep and
one-sweep slab launches and the per-half kernels; on the batched 32^3
lattices the one-launch and per-half bit-plane sweeps and the byte layout's
resident kernel -- independent implementations of the same trajectory must
reach identical spins, daemons and energies.
"""
import hashlib

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2506_16240_amd import micsa as M
from paper_2506_16240_amd import workloads as W

pytestmark = pytest.mark.gpu

# (shape, layout, kernel option): each reaches a different sweep path
PATHS = [
    ((16, 16, 16, 1, 2), M.LAYOUT_BYTE, M.KERNEL_AUTO),      # resident kernel
    ((16, 6, 10, 2, 3), M.LAYOUT_BYTE, M.KERNEL_SIMPLE),     # per-half kernels
    ((64, 8, 6, 1, 2), M.LAYOUT_BYTE, M.KERNEL_SLAB),        # slab, two sweeps per launch
    ((160, 12, 8, 1, 2), M.LAYOUT_BYTE, M.KERNEL_FUSED),     # fused byte sweep
    ((128, 6, 8, 2, 1), M.LAYOUT_BYTE, M.KERNEL_MULTISPIN),  # multispin planes
    ((8, 8, 8, 70, 2), M.LAYOUT_BITPLANE, M.KERNEL_AUTO),    # bit planes, two words of lanes
]
IDS = ["resident", "per-half", "slab", "fused", "multispin", "bitplane"]


def _lattice(shape, layout, kernel, seed):
    Lx, Ly, Lz, S, R = shape
    g = M.Lattice(Lx, Ly, Lz, S, R, seed, layout=layout)
    g.set_option(M.OPT_SWEEP_KERNEL, kernel)
    return g


@pytest.mark.parametrize("algo", [M.ALGO_MICSA, M.ALGO_HEATBATH], ids=["micsa", "heatbath"])
@pytest.mark.parametrize("shape,layout,kernel", PATHS, ids=IDS)
def test_device_log_equals_host_log_and_oracle(shape, layout, kernel, algo):
    if layout == M.LAYOUT_BITPLANE and algo != M.ALGO_MICSA:
        pytest.skip("the bit-plane layout runs MicSA only")
    Lx, Ly, Lz, S, R = shape
    stride, L = 4, S * R  # 27 sweeps: 6 rows and a tail of 3 unlogged sweeps
    gs, os_ = M.Schedule(M.SCHED_LINEAR, 2.5, 0.4, 60, 5), O.Schedule(O.SCHED_LINEAR, 2.5, 0.4, 60, 5)
    a = _lattice(shape, layout, kernel, 0x10C)
    b = _lattice(shape, layout, kernel, 0x10C)
    o = O.Lattice(Lx, Ly, Lz, S, R, 0x10C)
    for g in (a, b):
        g.set_schedule(gs)
    dev = torch.device("cuda:0")
    # three calls (27 + 27 + 6 sweeps of the 60-sweep schedule): both logs,
    # the energy log alone, the daemon log alone
    for n, want_e, want_d in ((27, True, True), (27, True, False), (6, False, True)):
        rows = n // stride
        E_d = torch.full((rows, L), -7, dtype=torch.int64, device=dev) if want_e else None
        D_d = torch.full((rows, L), -7, dtype=torch.int64, device=dev) if want_d else None
        torch.cuda.synchronize()
        a.sweep_logged_d(algo, n, stride, E_d, D_d)
        a.sync()
        Eh, Dh = b.sweep_logged(algo, n, stride)
        Eo, Do = o.run(algo, os_, n, stride)
        if want_e:
            got = E_d.cpu().numpy()
            assert np.array_equal(got, Eh) and np.array_equal(got, Eo), (n, got, Eo)
        if want_d:
            got = D_d.cpu().numpy()
            assert np.array_equal(got, Dh) and np.array_equal(got, Do), (n, got, Do)
    assert np.array_equal(a.spins(), o.sigma) and np.array_equal(a.daemons(), o.m)
    assert a.counters() == b.counters()
    a.close()
    b.close()


def test_device_log_without_rows_only_sweeps():
    """stride > n: no row, no write; the sweeps still run."""
    g = M.Lattice(16, 6, 10, 1, 1, 5)
    o = O.Lattice(16, 6, 10, 1, 1, 5)
    g.set_schedule(M.Schedule(M.SCHED_CONST, 1.0, 1.0, 20, 3))
    g.sweep_logged_d(M.ALGO_MICSA, 5, 8, None, None)
    o.run(O.ALGO_MICSA, O.Schedule(O.SCHED_CONST, 1.0, 1.0, 20, 3), 5, 0)
    assert np.array_equal(g.spins(), o.sigma) and np.array_equal(g.daemons(), o.m)
    with pytest.raises(M.MicsaError):
        g.sweep_logged_d(M.ALGO_MICSA, 5, 0, None, None)
    g.close()


def _digest(g, tally=True):
    """Spins, daemons, energy, daemon energy and (where the path keeps one)
    the incremental tally."""
    h = hashlib.sha256()
    parts = [g.spins(), g.daemons(), g.energy(), g.daemon_energy()]
    if tally:
        parts.append(g.energy_tally())
    for x in parts:
        h.update(np.ascontiguousarray(x).tobytes())
    return h.hexdigest()


def test_anneal_L512_state_hashes_at_powers_of_ten():
    """The whole 10^4-sweep anneal at 512^3: multispin (automatic launch
    shape), fused byte and per-half kernels agree at k = 10, 100, 1000,
    10000, and the tally equals the from-scratch energy at each point."""
    w = W.ANNEAL_L512
    marks = [10, 100, 1000, 10000]
    assert marks[-1] == w.n_sweeps
    hashes = {}
    for name, kernel in (("multispin", M.KERNEL_AUTO), ("fused", M.KERNEL_FUSED), ("per-half", M.KERNEL_SIMPLE)):
        g = M.Lattice(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
        g.set_option(M.OPT_SWEEP_KERNEL, kernel)
        if kernel == M.KERNEL_AUTO:
            assert g.kernel_name(M.ALGO_MICSA).startswith("k_msc_sweep")
        g.set_schedule(M.Schedule(w.kind, w.T0, w.T1, w.n_sweeps, w.period))
        k, got = 0, []
        for mark in marks:
            g.sweep(M.ALGO_MICSA, mark - k)
            k = mark
            assert np.array_equal(g.energy_tally(), g.energy()), (name, mark)
            got.append(_digest(g))
        print(f"[hash] {name}: " + " ".join(f"k={m}:{d[:12]}" for m, d in zip(marks, got)), flush=True)
        hashes[name] = got
        g.close()
    assert hashes["multispin"] == hashes["fused"] == hashes["per-half"]


def _run_hashes(w, marks, layout, kernel):
    g = M.Lattice(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed, layout=layout)
    g.set_option(M.OPT_SWEEP_KERNEL, kernel)
    g.set_schedule(M.Schedule(w.kind, w.T0, w.T1, w.n_sweeps, w.period))
    name = g.kernel_name(M.ALGO_MICSA)
    k, got = 0, []
    for mark in marks:
        g.sweep(M.ALGO_MICSA, mark - k)
        k = mark
        got.append(_digest(g, tally=False))  # the bit-plane per-half kernels keep no tally
    g.close()
    return name, got


def test_quench_L64_state_hashes_at_powers_of_ten():
    """Configuration 2 over its whole 10^5-sweep schedule: the two-sweep slab
    launch (the library's choice), the one-sweep slab launch and the per-half
    kernels agree at k = 10 .. 10^5."""
    w = W.QUENCH_L64
    marks = [10, 100, 1000, 10000, 100000]
    assert marks[-1] == w.n_sweeps
    runs = {}
    for kernel in (M.KERNEL_AUTO, M.KERNEL_SLAB, M.KERNEL_SIMPLE):
        name, got = _run_hashes(w, marks, M.LAYOUT_BYTE, kernel)
        runs[name] = got
        print(f"[hash] {name}: " + " ".join(f"k={m}:{d[:12]}" for m, d in zip(marks, got)), flush=True)
    assert "k_micsa_slab2" in runs and "k_micsa_half" in runs
    assert len({tuple(v) for v in runs.values()}) == 1


def test_batched_L32_state_hashes_at_powers_of_ten():
    """Configuration 3 over its whole 10^4-sweep schedule: the one-launch
    bit-plane sweep (the library's choice), the bit-plane per-half kernels
    and the byte layout's resident kernel agree at k = 10 .. 10^4."""
    w = W.BATCHED_L32
    marks = [10, 100, 1000, 10000]
    assert marks[-1] == w.n_sweeps
    runs = []
    for layout, kernel in ((M.LAYOUT_BITPLANE, M.KERNEL_AUTO), (M.LAYOUT_BITPLANE, M.KERNEL_SIMPLE),
                           (M.LAYOUT_BYTE, M.KERNEL_AUTO)):
        name, got = _run_hashes(w, marks, layout, kernel)
        runs.append((name, got))
        print(f"[hash] {name}: " + " ".join(f"k={m}:{d[:12]}" for m, d in zip(marks, got)), flush=True)
    assert [n for n, _ in runs] == ["kb_sweep", "kb_micsa_half", "k_resident<0>"]
    assert runs[0][1] == runs[1][1] == runs[2][1]
