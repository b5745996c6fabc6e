"""GPU parity: the HIP path through the C ABI against the CPU oracle.

MicSA and the heat bath are integer dynamics with a fixed random-number
specification, so there is exactly one correct trajectory: parity is bit
equality of every logged energy, of the final spins and daemons, and of
the couplings.  Shapes span several words per row, ragged (non power of
two) sides, the minimum sides, several samples and replicas, and the
configurations' own sizes (full size where the oracle can follow; the
first sweeps otherwise).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2506_16240_amd import micsa as M
from paper_2506_16240_amd import workloads as W

pytestmark = pytest.mark.gpu


def pair(Lx, Ly, Lz, S=1, R=1, seed=1):
    return M.Lattice(Lx, Ly, Lz, S, R, seed), O.Lattice(Lx, Ly, Lz, S, R, seed)


def scheds(kind, T0, T1, n, P, table=None):
    return M.Schedule(kind, T0, T1, n, P, table), O.Schedule(kind, T0, T1, n, P, table)


def same_state(g, o):
    assert np.array_equal(g.spins(), o.sigma), "spins differ"
    assert np.array_equal(g.daemons(), o.m), "daemons differ"


SHAPES = [
    (8, 8, 8, 1, 1),      # one 4-site word pair per row
    (8, 2, 2, 1, 2),      # minimum sides
    (16, 6, 10, 2, 3),    # several samples and replicas, ragged y/z
    (24, 4, 6, 1, 2),     # three words per row
    (40, 10, 6, 3, 1),    # ragged x (5 words per row)
    (32, 32, 32, 2, 2),
]


@pytest.mark.parametrize("shape", SHAPES)
def test_initial_state_matches_oracle(shape):
    g, o = pair(*shape, seed=0xABCDEF12345)
    assert np.array_equal(g.couplings(), o.J)
    same_state(g, o)
    E = o.energy()
    assert np.array_equal(g.energy(), E)
    assert np.array_equal(g.energy_tally(), E)
    assert np.array_equal(g.daemon_energy(), np.zeros_like(E))


def test_thresholds_bitexact():
    g, _ = pair(8, 8, 8)
    cases = [scheds(M.SCHED_CONST, T, T, 100, 10) for T in (0.05, 0.1, 0.2, 0.7, 1.1019, 1.5, 3.0, 1e6)]
    cases.append(scheds(M.SCHED_LINEAR, 3.0, 0.2, 10000, 20))
    cases.append(scheds(M.SCHED_LINEAR, 3.0, 0.1, 2000, 10))
    cases.append(scheds(M.SCHED_TABLE, 0, 0, 30, 10, np.array([2.5, 0.9, 0.31])))
    cases.append(scheds(M.SCHED_LINEAR, 2.0, 0.5, 1000, M.REFRESH_LOG2))
    for gs, os_ in cases:
        g.set_schedule(gs)
        for rho in range(os_.refresh_count()):
            T = os_.temperature(rho)
            assert np.array_equal(g.thresholds(rho), O.daemon_thresholds(T)), (gs, rho)
            assert np.array_equal(g.heatbath_thresholds(rho), O.heatbath_thresholds(T)), (gs, rho)
            assert np.array_equal(g.metropolis_thresholds(rho), O.metropolis_thresholds(T)), (gs, rho)


@pytest.mark.parametrize("kernel", [M.KERNEL_SIMPLE, M.KERNEL_RESIDENT])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("algo", [M.ALGO_MICSA, M.ALGO_HEATBATH, M.ALGO_METROPOLIS])
def test_trajectory_matches_oracle(shape, algo, kernel):
    g, o = pair(*shape, seed=77)
    g.set_option(M.OPT_SWEEP_KERNEL, kernel)
    n = 37
    gs, os_ = scheds(M.SCHED_LINEAR, 2.5, 0.4, n, 6)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(algo, n, 1)
    Eo, Do = o.run(algo, os_, n, 1)
    assert np.array_equal(Eg, Eo)
    if algo == M.ALGO_MICSA:
        assert np.array_equal(Dg, Do)
    same_state(g, o)
    assert np.array_equal(g.energy_tally(), o.energy())
    assert g.counters()[0] == n


def test_log2_refresh_schedule_matches_oracle():
    g, o = pair(16, 8, 6, 1, 2, seed=5)
    n = 70
    gs, os_ = scheds(M.SCHED_CONST, 0.9, 0.9, n, M.REFRESH_LOG2)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, n, 1)
    Eo, Do = o.run(O.ALGO_MICSA, os_, n, 1)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    same_state(g, o)


@pytest.mark.parametrize("kernel", [M.KERNEL_AUTO, M.KERNEL_SIMPLE])
def test_paramagnet_L16_full_length(kernel):
    """L = 16, T = 1.5, refresh every 10 sweeps, 1000 sweeps, energy logged per
    sweep: bit-exact, and H^EA + H^aux conserved between refreshes."""
    w = W.PARAMAGNET_L16
    g, o = pair(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
    g.set_option(M.OPT_SWEEP_KERNEL, kernel)
    gs, os_ = scheds(w.kind, w.T0, w.T1, w.n_sweeps, w.period)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, w.n_sweeps, 1)
    Eo, Do = o.run(O.ALGO_MICSA, os_, w.n_sweeps, 1)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    same_state(g, o)
    tot = (Eg + Dg)[:, 0]
    for r in range(1, w.n_sweeps):
        if r % w.period != 0:  # sweep r did not start with a refresh
            assert tot[r] == tot[r - 1]
    assert np.array_equal(g.energy_tally(), g.energy())


def test_resident_chunks_and_log_strides():
    """Resident launches split long runs into chunks; logs and state must not
    depend on where the chunks fall."""
    shape = (16, 8, 8, 2, 2)
    n = 4500  # crosses two chunk boundaries
    for stride in (1, 7, 1000):
        g, o = pair(*shape, seed=8)
        g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_RESIDENT)
        gs, os_ = scheds(M.SCHED_LINEAR, 3.0, 0.3, n, 9)
        g.set_schedule(gs)
        Eg, Dg = g.sweep_logged(M.ALGO_MICSA, n, stride)
        Eo, Do = o.run(O.ALGO_MICSA, os_, n, stride)
        assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
        same_state(g, o)
        assert np.array_equal(g.energy_tally(), o.energy())


def test_quench_L64_shape():
    """L = 64, 1 sample x 2 replicas, T = 0.7: MicSA and heat bath from the same
    seed, energies, daemon energies and the replica overlap."""
    w = W.QUENCH_L64
    n = 120
    for algo in (M.ALGO_MICSA, M.ALGO_HEATBATH, M.ALGO_METROPOLIS):
        g, o = pair(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
        gs, os_ = scheds(w.kind, w.T0, w.T1, w.n_sweeps, w.period)
        g.set_schedule(gs)
        Eg, Dg = g.sweep_logged(algo, n, 10)
        Eo, Do = o.run(algo, os_, n, 10)
        assert np.array_equal(Eg, Eo)
        if algo == M.ALGO_MICSA:
            assert np.array_equal(Dg, Do)
        assert np.array_equal(g.overlap(0, 1), o.overlap(0, 1))
        assert np.array_equal(g.overlap(1, 0), o.overlap(1, 0))
        same_state(g, o)


SLAB_SHAPES = [(8, 2, 2, 1, 1), (8, 4, 6, 2, 3), (24, 6, 10, 1, 2), (64, 16, 4, 3, 1), (128, 64, 6, 1, 1),
               (40, 10, 8, 2, 2),
               (64, 8, 64, 1, 4)]  # 256 planes: a full grid keeps one sweep per launch


def slab_kernel(shape):
    """The slab launch the library picks: two sweeps per launch while the
    lattices have fewer planes than the device has compute units."""
    Lx, Ly, Lz, S, R = shape
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    return "k_micsa_slab2" if S * R * Lz < cus else "k_micsa_slab"


@pytest.mark.parametrize("ahead", [1, 0], ids=["drawn-ahead", "drawn-in-kernel"])
@pytest.mark.parametrize("shape", SLAB_SHAPES)
def test_slab_sweep_matches_oracle(shape, ahead):
    """The one-launch slab sweep (a z plane per work-group, neighbour planes
    recomputed): minimum sides (one word per row, planes that wrap onto a
    side of 2), several samples and replicas, ragged words per row, a plane
    of 1024 words, a grid of one plane per compute unit; refresh levels
    drawn ahead on the side stream or in the kernel; refresh every sweep and
    every fourth; logged energies, tally and state against the oracle."""
    g, o = pair(*shape, seed=0x51AB)
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_SLAB)
    g.set_option(M.OPT_DRAW_AHEAD, ahead)
    assert g.kernel_name(M.ALGO_MICSA) == slab_kernel(shape)
    for P, n in ((1, 5), (4, 13)):
        gs, os_ = scheds(M.SCHED_LINEAR, 2.5, 0.4, 100, P)
        g.set_schedule(gs)
        o_k = g.counters()[0]
        Eg, Dg = g.sweep_logged(M.ALGO_MICSA, n, 1)
        Eo, Do = o.run(O.ALGO_MICSA, os_, n, 1)
        assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do), (P, o_k)
        same_state(g, o)
        assert np.array_equal(g.energy_tally(), o.energy())
    # long calls: two sweeps per launch (refresh on the first, the second or
    # both sweeps of a pair; a call starting at odd k; a last single sweep)
    for P, n in ((3, 11), (1, 6), (3, 9)):
        gs, os_ = scheds(M.SCHED_LINEAR, 2.5, 0.4, 100, P)
        g.set_schedule(gs)
        g.sweep(M.ALGO_MICSA, n)
        o.run(O.ALGO_MICSA, os_, n, 0)
        same_state(g, o)
        assert np.array_equal(g.energy_tally(), o.energy())
    g.sweep(M.ALGO_HEATBATH, 2)  # the baselines keep their own kernels on the same context
    o.run(O.ALGO_HEATBATH, os_, 2)
    same_state(g, o)


@pytest.mark.parametrize("ahead", [1, 0], ids=["drawn-ahead", "drawn-in-kernel"])
def test_quench_L64_slab_1000_sweeps(ahead):
    """Configuration 2 (L = 64, two replicas, T = 0.7, refresh every 10) on the
    library's own kernel choice, the two-sweep slab launch, for 1000 sweeps in
    long calls, refresh levels drawn ahead (the default) or in the kernel:
    state, energies, daemon energies, tally and overlap equal the oracle's."""
    w = W.QUENCH_L64
    g, o = pair(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
    g.set_option(M.OPT_DRAW_AHEAD, ahead)
    assert g.kernel_name(M.ALGO_MICSA) == "k_micsa_slab2"
    gs, os_ = scheds(w.kind, w.T0, w.T1, w.n_sweeps, w.period)
    g.set_schedule(gs)
    for n in (333, 666, 1):  # pairs with the refresh first, then (from k = 333) second in the pair
        g.sweep(M.ALGO_MICSA, n)
        o.run(O.ALGO_MICSA, os_, n, 0)
    same_state(g, o)
    E = o.energy()
    assert np.array_equal(g.energy(), E) and np.array_equal(g.energy_tally(), E)
    assert np.array_equal(g.daemon_energy(), o.daemon_energy())
    assert np.array_equal(g.overlap(0, 1), o.overlap(0, 1))


def test_batched_L32_shape():
    """L = 32, 256 samples x 2 replicas in one context (byte layout)."""
    w = W.BATCHED_L32
    n = 12
    g, o = pair(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
    gs, os_ = scheds(w.kind, w.T0, w.T1, w.n_sweeps, w.period)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, n, 4)
    Eo, Do = o.run(O.ALGO_MICSA, os_, n, 4)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    assert np.array_equal(g.overlap(0, 1), o.overlap(0, 1))
    same_state(g, o)


@pytest.mark.parametrize("prefetch,temporal,kernel", [(1, 2, M.KERNEL_AUTO), (2, 1, M.KERNEL_AUTO),
                                                      (1, 2, M.KERNEL_MULTISPIN)])
def test_anneal_L512_first_sweeps_full_size(prefetch, temporal, kernel):
    """L = 512 (134M spins), linear 3.0 -> 0.2 over 10^4 sweeps, refresh every 20:
    the first 21 sweeps (two refreshes) bit-exact at full size, with the
    fused sweep's benchmark tile, two sweeps per pass (logging every 7
    sweeps: pairs and a single sweep per call) and one sweep per pass at
    both prefetch depths, and on the multispin planes."""
    w = W.ANNEAL_L512
    n = 21
    g, o = pair(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
    g.set_option(M.OPT_SWEEP_KERNEL, kernel)
    g.set_option(M.OPT_TILE_Y, 32)
    g.set_option(M.OPT_TILE_Z, 32)
    g.set_option(M.OPT_PREFETCH, prefetch)
    g.set_option(M.OPT_TEMPORAL, temporal)
    gs, os_ = scheds(w.kind, w.T0, w.T1, w.n_sweeps, w.period)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, n, 7)
    Eo, Do = o.run(O.ALGO_MICSA, os_, n, 7)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    same_state(g, o)
    assert np.array_equal(g.energy_tally(), g.energy())


@pytest.mark.parametrize("algo", [M.ALGO_MICSA, M.ALGO_WALKERS])
def test_anneal_L512_default_launch_full_size(algo):
    """The 512^3 anneal exactly as the benchmark times it: no launch option
    (the library's own choice: two sweeps per pass over the multispin planes
    with the automatic 24-row, 16-plane tile and its ragged last y tile,
    z-band XCD order over the z tiles, refresh levels drawn ahead on the
    side stream; walkers wander between the pass's two sweeps and owe the
    second's to the next call), 41 sweeps in ONE call (refreshes before
    sweeps 0, 20 and 40, two of them drawn ahead inside the call), then 3
    more in a second call.  Spins, daemons, energy, daemon energy and the
    tally equal the oracle's bit for bit."""
    w = W.ANNEAL_L512
    g, o = pair(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
    gs, os_ = scheds(w.kind, w.T0, w.T1, w.n_sweeps, w.period)
    g.set_schedule(gs)
    oalgo = O.ALGO_MICSA if algo == M.ALGO_MICSA else O.ALGO_WALKERS
    for n in (41, 3):
        g.sweep(algo, n)
        o.run(oalgo, os_, n, 0)
        assert g.kernel_name(algo) == "k_msc_sweep_multi"
        same_state(g, o)
        E = o.energy()
        assert np.array_equal(g.energy(), E)
        assert np.array_equal(g.daemon_energy(), o.daemon_energy())
        assert np.array_equal(g.energy_tally(), E)


@pytest.mark.parametrize("ty,tz", [(0, 0), (24, 16)])
def test_anneal_L512_two_sweep_pass_full_size(ty, tz):
    """The 512^3 anneal with two multispin sweeps per pass (the automatic
    tile and the 24 x 16 tile), in calls of 41, 19 and 2 sweeps: a refresh
    drawn inside the first sweep of the first call (one-sweep kernel), the
    refreshes at sweeps 20 and 40 on the second sweep of a pass (drawn ahead,
    read by the pass), the refresh at 60 on the first sweep of a pass (drawn
    during the call before), and a last odd sweep of a call on the one-sweep
    kernel.  Spins, daemons, energy, daemon energy and tally equal the
    oracle's bit for bit after every call."""
    w = W.ANNEAL_L512
    g, o = pair(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
    g.set_option(M.OPT_MSC_PASS, 2)
    if ty:
        g.set_option(M.OPT_TILE_Y, ty)
        g.set_option(M.OPT_TILE_Z, tz)
    gs, os_ = scheds(w.kind, w.T0, w.T1, w.n_sweeps, w.period)
    g.set_schedule(gs)
    for n in (41, 19, 2):
        g.sweep(M.ALGO_MICSA, n)
        o.run(O.ALGO_MICSA, os_, n, 0)
        assert g.kernel_name(M.ALGO_MICSA) == "k_msc_sweep_multi"
        same_state(g, o)
        E = o.energy()
        assert np.array_equal(g.energy(), E)
        assert np.array_equal(g.daemon_energy(), o.daemon_energy())
        assert np.array_equal(g.energy_tally(), E)


@pytest.mark.parametrize("algo", [M.ALGO_HEATBATH, M.ALGO_METROPOLIS])
def test_anneal_L512_baseline_first_sweeps_full_size(algo):
    """The heat-bath and Metropolis baselines on the 512^3 lattice: first 6
    sweeps bit-exact."""
    w = W.ANNEAL_L512
    n = 6
    g, o = pair(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
    gs, os_ = scheds(w.kind, w.T0, w.T1, w.n_sweeps, w.period)
    g.set_schedule(gs)
    Eg, _ = g.sweep_logged(algo, n, 3)
    Eo, _ = o.run(algo, os_, n, 3)
    assert np.array_equal(Eg, Eo)
    assert np.array_equal(g.spins(), o.sigma)
    assert np.array_equal(g.energy_tally(), g.energy())


def test_written_state_is_swept_identically():
    """Injected spins and daemons (no refresh in between) evolve identically."""
    g, o = pair(16, 8, 8, 2, 2, seed=3)
    gs, os_ = scheds(M.SCHED_CONST, 1.0, 1.0, 100, 1000)
    g.set_schedule(gs)
    g.sweep(M.ALGO_MICSA, 3)
    o.run(O.ALGO_MICSA, os_, 3, 0)
    rng = np.random.default_rng(4)
    o.sigma[:] = rng.integers(0, 2, o.sigma.shape, dtype=np.uint8)
    o.m[:] = rng.integers(0, 4, o.m.shape, dtype=np.uint8)
    o.tally = o.energy()
    g.write_spins(o.sigma)
    g.write_daemons(o.m)
    same_state(g, o)
    assert np.array_equal(g.energy_tally(), o.energy())
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, 10, 1)
    Eo, Do = o.run(O.ALGO_MICSA, os_, 10, 1)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    # no refresh: total energy is exactly conserved over all 10 sweeps
    assert len(set((Eg + Dg)[:, 0])) == 1
    same_state(g, o)


@pytest.mark.parametrize("layout", [M.LAYOUT_BYTE, M.LAYOUT_BITPLANE])
@pytest.mark.parametrize("algo", [M.ALGO_MICSA, M.ALGO_HEATBATH, M.ALGO_METROPOLIS])
def test_graph_replays_match_eager_launches(layout, algo):
    """Replayed graphs (16 sweeps each, device sweep counter) give the same bits
    as eager launches and as the oracle, over several calls with eager work
    and reads in between and a refresh period that does not divide 16."""
    if layout == M.LAYOUT_BITPLANE and algo != M.ALGO_MICSA:
        pytest.skip("the canonical baselines run in the byte layout")
    shape = (64, 8, 6, 3, 2)  # byte: neither resident (forced simple) nor fused
    res = []
    for graphs in (1, 0):
        g = M.Lattice(*shape, seed=515, layout=layout)
        if layout == M.LAYOUT_BYTE:
            g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_SIMPLE)
        g.set_option(M.OPT_GRAPHS, graphs)
        g.set_schedule(M.Schedule(M.SCHED_LINEAR, 2.6, 0.3, 200, 7))
        E = []
        for n in (40, 3, 33, 16, 50):
            g.sweep(algo, n)
            E.append(g.energy())  # eager reduction between replays
        res.append((np.array(E), g.spins(), g.daemons(), g.counters()))
        g.close()
    for a, b in zip(res[0][:3], res[1][:3]):
        assert np.array_equal(a, b)
    assert res[0][3] == res[1][3] == (142, 20)
    o = O.Lattice(*shape, seed=515)
    o.run(algo, O.Schedule(O.SCHED_LINEAR, 2.6, 0.3, 200, 7), 142, 0)
    assert np.array_equal(res[0][1], o.sigma)
    assert np.array_equal(res[0][0][-1], o.energy())


@pytest.mark.parametrize("shape,kernel", [((16, 6, 10, 2, 2), M.KERNEL_AUTO), ((8, 2, 2, 1, 1), M.KERNEL_SIMPLE),
                                          ((64, 8, 6, 1, 2), M.KERNEL_FUSED), ((96, 8, 4, 1, 1), M.KERNEL_SIMPLE)])
def test_walkers_match_oracle(shape, kernel):
    """One walker per site, forward-X wandering after every sweep (Sec. 2.6)."""
    g, o = pair(*shape, seed=4321)
    g.set_option(M.OPT_SWEEP_KERNEL, kernel)
    n = 31
    gs, os_ = scheds(M.SCHED_LINEAR, 2.0, 0.5, n, 4)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(M.ALGO_WALKERS, n, 1)
    Eo, Do = o.run(O.ALGO_WALKERS, os_, n, 1)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    same_state(g, o)
    assert np.array_equal(g.energy_tally(), o.energy())


@pytest.mark.parametrize("shape", [(128, 8, 6, 1, 2), (96, 6, 4, 1, 1), (64, 4, 8, 2, 1)])
@pytest.mark.parametrize("prefetch,temporal", [(1, 1), (2, 1), (1, 2)])
def test_walkers_fused_wander_on_load(shape, prefetch, temporal):
    """Walkers on the fused sweeps: each timestep's forward-X wandering is
    applied by the next sweep as it loads the daemons, and inside the
    two-sweep kernel between its two sweeps (rows of 2 or 4 chunks; rows of
    3 chunks fall back to the one-sweep kernel).  Stretches of up to 8
    sweeps between refreshes, pairs and single sweeps in turn, a wandering
    still owed when the daemons are read back, and a switch to daemons
    (which applies it first)."""
    g, o = pair(*shape, seed=777)
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_FUSED)
    g.set_option(M.OPT_PREFETCH, prefetch)
    g.set_option(M.OPT_TEMPORAL, temporal)
    gs, os_ = scheds(M.SCHED_LINEAR, 2.2, 0.4, 60, 9)
    g.set_schedule(gs)
    two = temporal == 2 and 64 % (shape[0] // 32) == 0
    assert g.kernel_name(M.ALGO_WALKERS) == ("k_micsa_sweep2_fused" if two else "k_micsa_sweep_fused")
    for n in (13, 1, 2, 3):
        g.sweep(M.ALGO_WALKERS, n)
        o.run(O.ALGO_WALKERS, os_, n)
    same_state(g, o)
    g.sweep(M.ALGO_WALKERS, 20)
    o.run(O.ALGO_WALKERS, os_, 20)
    assert np.array_equal(g.energy(), o.energy())
    g.sweep(M.ALGO_MICSA, 7)
    o.run(O.ALGO_MICSA, os_, 7)
    same_state(g, o)
    assert np.array_equal(g.energy_tally(), o.energy())


MSC_SHAPES = [(128, 4, 4, 1, 1), (128, 2, 2, 1, 1), (128, 6, 2, 2, 3), (384, 4, 6, 1, 2), (256, 8, 6, 2, 1),
              (128, 70, 36, 1, 1),  # several tiles along z
              (512, 50, 4, 1, 1)]  # automatic tile of 44 rows: a second tile of 6 along y


@pytest.mark.parametrize("fused,ahead", [(1, 1), (1, 0), (0, 1)], ids=["one-launch", "one-launch-in-sweep-draw",
                                                                       "per-half"])
@pytest.mark.parametrize("shape", MSC_SHAPES)
def test_multispin_matches_oracle(shape, fused, ahead):
    """Multispin coding (Sec. 2.5): 64 sites of a row per word, the Creutz
    move bit-sliced; one launch per sweep marching along z (rings of rows
    and planes that wrap onto small sides; refresh levels drawn ahead on the
    side stream or inside the sweep) or one per half sweep.  Every logged
    energy (one pack/unpack per sweep), then a long call (one pack, many
    sweeps, one unpack), against the oracle; minimum sides, several samples
    and replicas, three words per row."""
    g, o = pair(*shape, seed=0x77AA)
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_MULTISPIN)
    g.set_option(M.OPT_MSC_FUSED, fused)
    g.set_option(M.OPT_MSC_PASS, 1)  # one sweep per launch (two per pass: test_multispin_two_sweeps_per_pass...)
    g.set_option(M.OPT_DRAW_AHEAD, ahead)
    assert g.kernel_name(M.ALGO_MICSA) == ("k_msc_sweep" if fused else "k_msc_half")
    gs, os_ = scheds(M.SCHED_LINEAR, 2.4, 0.3, 60, 3)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, 9, 1)
    Eo, Do = o.run(O.ALGO_MICSA, os_, 9, 1)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    same_state(g, o)
    g.sweep(M.ALGO_MICSA, 31)
    o.run(O.ALGO_MICSA, os_, 31)
    same_state(g, o)
    assert np.array_equal(g.energy_tally(), o.energy())
    assert np.array_equal(g.couplings(), o.J)
    # the other algorithms keep the fused path on the same context
    g.sweep(M.ALGO_HEATBATH, 3)
    o.run(O.ALGO_HEATBATH, os_, 3)
    same_state(g, o)


@pytest.mark.parametrize("ahead", [1, 0], ids=["drawn-ahead", "drawn-in-sweep"])
def test_multispin_planes_live_between_calls(ahead):
    """A multispin call leaves its planes live and (with the draw ahead) the
    levels of the next call's first refresh drawn: calls that end between
    refreshes and start at a drawn one, reads between calls, a heat-bath
    call, a short call on the byte path, walkers, a schedule change (the
    drawn levels are dropped), a checkpoint into a fresh context, the
    written state of write_spins; every state against the oracle."""
    shape = (256, 6, 4, 1, 2)
    g, o = pair(*shape, seed=0x11FE)
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_MULTISPIN)
    g.set_option(M.OPT_DRAW_AHEAD, ahead)
    gs, os_ = scheds(M.SCHED_LINEAR, 2.6, 0.3, 200, 5)
    g.set_schedule(gs)

    def both(algo, n):
        g.sweep(algo, n)
        o.run(algo, os_, n, 0)

    both(M.ALGO_MICSA, 12)  # ends between refreshes; the refresh at 15 is drawn ahead
    both(M.ALGO_MICSA, 8)   # starts at 12, uses it
    assert np.array_equal(g.energy(), o.energy())
    both(M.ALGO_MICSA, 10)
    same_state(g, o)
    both(M.ALGO_HEATBATH, 2)  # the byte arrays, then the planes packed again
    both(M.ALGO_MICSA, 9)
    both(M.ALGO_MICSA, 3)    # a short call
    both(M.ALGO_MICSA, 16)
    both(M.ALGO_WALKERS, 12)
    both(M.ALGO_MICSA, 10)
    assert np.array_equal(g.energy_tally(), o.energy())
    same_state(g, o)
    gs2, os2 = scheds(M.SCHED_LINEAR, 1.9, 0.5, 200, 5)  # other temperatures: drawn levels dropped
    g.set_schedule(gs2)
    os_ = os2
    both(M.ALGO_MICSA, 13)
    both(M.ALGO_MICSA, 11)
    image = g.save()
    h = M.Lattice(*shape, seed=0x11FE)
    h.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_MULTISPIN)
    h.load(image)
    both(M.ALGO_MICSA, 9)
    h.sweep(M.ALGO_MICSA, 9)
    for x in (g, h):
        same_state(x, o)
        assert np.array_equal(x.energy(), o.energy())
    spins = o.sigma.copy()
    spins[0, 0, :7] ^= 1
    g.write_spins(spins)
    o.sigma = spins
    both(M.ALGO_MICSA, 14)
    same_state(g, o)
    assert np.array_equal(g.energy_tally(), o.energy())
    h.close()
    g.close()


@pytest.mark.parametrize("passes", [1, 2], ids=["one-sweep", "two-sweep"])
@pytest.mark.parametrize("shape", [(128, 4, 4, 1, 1), (256, 6, 4, 1, 2), (384, 4, 6, 2, 1), (512, 50, 4, 1, 1)])
def test_multispin_walkers_match_oracle(shape, passes):
    """Walkers (gamma = 1, forward-X wandering after every timestep, Sec.
    2.6) on the one-launch multispin sweep: each sweep applies the previous
    timestep's wandering as it loads the levels (one or three words per
    row), the last one is left owed to the byte state; and two sweeps per
    pass, the first sweep's wandering applied between them (rows of one,
    two and four words; three words per row fall back to one sweep per
    launch).  Calls of walkers and daemons in turn, the daemons read back in
    between, single sweeps and long calls, against the oracle."""
    g, o = pair(*shape, seed=0x77AB)
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_MULTISPIN)
    g.set_option(M.OPT_MSC_PASS, passes)
    W = shape[0] // 128
    expect = "k_msc_sweep_multi" if passes == 2 and 64 % W == 0 else "k_msc_sweep"
    assert g.kernel_name(M.ALGO_WALKERS) == expect
    gs, os_ = scheds(M.SCHED_LINEAR, 2.4, 0.3, 90, 7)
    g.set_schedule(gs)
    for algo, oalgo, n in ((M.ALGO_WALKERS, O.ALGO_WALKERS, 12), (M.ALGO_WALKERS, O.ALGO_WALKERS, 1),
                           (M.ALGO_MICSA, O.ALGO_MICSA, 9), (M.ALGO_WALKERS, O.ALGO_WALKERS, 23)):
        g.sweep(algo, n)
        o.run(oalgo, os_, n)
        same_state(g, o)
    g.sweep(M.ALGO_WALKERS, 15)
    o.run(O.ALGO_WALKERS, os_, 15)
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_FUSED)  # the owed wandering passes to the byte sweeps
    g.sweep(M.ALGO_WALKERS, 5)
    o.run(O.ALGO_WALKERS, os_, 5)
    same_state(g, o)
    assert np.array_equal(g.energy_tally(), o.energy())


def test_multispin_launch_shapes_give_the_same_bits():
    """The one-launch multispin sweep at every tile shape (one row or plane
    per tile, odd and even step counts, tiles that do not fill a wave, a
    last tile along y shorter than the others; tiles in plain or XCD order),
    with the refresh levels drawn inside the sweep or ahead of it on the
    side stream, agrees bit for bit with the per-half kernels, for daemons
    and walkers."""
    shape = (256, 12, 6, 1, 2)
    ref = None
    variants = [(0, 0, 0, 1, 1), (1, 0, 0, 0, 1), (1, 3, 2, 0, 1), (1, 5, 3, 0, 1), (1, 3, 3, 1, 0), (1, 1, 1, 1, 0)] + [
        (1, ty, tz, 1, 1) for ty in (1, 3, 4, 5, 7, 12) for tz in (1, 2, 3, 6)]  # 24, 72, 8 tiles: XCD order
    # two sweeps per pass (fused = 2 below): tiles of 1 .. 12 rows, z depths 1 .. 6, both tile orders
    variants += [(2, ty, tz, 1, xcd) for ty, tz, xcd in ((0, 0, 1), (1, 1, 1), (3, 2, 0), (5, 3, 1), (12, 6, 1),
                                                         (4, 1, 0))]
    for fused, ty, tz, ahead, xcd in variants:
        g = M.Lattice(*shape, seed=2025)
        g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_MULTISPIN)
        g.set_option(M.OPT_MSC_FUSED, min(fused, 1))
        g.set_option(M.OPT_MSC_PASS, 2 if fused == 2 else 1)
        g.set_option(M.OPT_DRAW_AHEAD, ahead)
        g.set_option(M.OPT_XCD_MAP, xcd)
        if ty:
            g.set_option(M.OPT_TILE_Y, ty)
            g.set_option(M.OPT_TILE_Z, tz)
        g.set_schedule(M.Schedule(M.SCHED_CONST, 0.8, 0.8, 60, 7))
        g.sweep(M.ALGO_MICSA, 23)  # refreshes at 0, 7, 14, 21
        got = [g.spins(), g.daemons(), g.energy_tally()]
        if fused:  # walkers run on the one-launch form only; compare them among its shapes
            g.sweep(M.ALGO_WALKERS, 17)
            got += [g.spins(), g.daemons()]
        if ref is None:
            ref = got
        elif fused and len(ref) == 3:
            ref_w = got[3:]
            assert all(np.array_equal(a, b) for a, b in zip(ref, got[:3])), (ty, tz, ahead, xcd)
            ref = ref + ref_w
        else:
            assert all(np.array_equal(a, b) for a, b in zip(ref, got)), (fused, ty, tz, ahead, xcd)
        g.close()


@pytest.mark.parametrize("shape,ty,tz", [((512, 50, 8, 1, 1), 0, 0), ((256, 12, 6, 1, 2), 5, 3),
                                         ((128, 6, 2, 2, 1), 0, 0), ((384, 10, 10, 1, 1), 2, 5)])
def test_multispin_two_sweeps_per_pass_match_oracle(shape, ty, tz):
    """Two sweeps per pass over the multispin planes (the default) against
    one sweep per pass and the oracle: calls that start at even and odd k,
    refreshes (period 5) on the first and on the second sweep of a pass,
    with the levels drawn ahead; a last odd sweep of a call on the one-sweep
    kernel; the ragged last y tile of the automatic 24-row tile."""
    gs, os_ = scheds(M.SCHED_LINEAR, 2.6, 0.4, 80, 5)
    o = O.Lattice(*shape, 0x2B)
    runs = {}
    for temporal in (2, 1):
        g = M.Lattice(*shape, 0x2B)
        g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_MULTISPIN)
        g.set_option(M.OPT_MSC_PASS, temporal)
        if ty:
            g.set_option(M.OPT_TILE_Y, ty)
            g.set_option(M.OPT_TILE_Z, tz)
        g.set_schedule(gs)
        states = []
        for n in (10, 9, 1, 14, 3):  # k = 0, 10, 19, 20, 34 at the starts
            g.sweep(M.ALGO_MICSA, n)
            if temporal == 2:
                o.run(O.ALGO_MICSA, os_, n, 0)
                same_state(g, o)
                assert np.array_equal(g.energy_tally(), o.energy())
            states.append((g.spins(), g.daemons(), g.energy_tally()))
        runs[temporal] = states
        g.close()
    for a, b in zip(runs[2], runs[1]):
        assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_multispin_tile_orders_give_the_same_bits():
    """Tiles in plain order, XCD by XCD, and in z bands per XCD (8 tiles
    along z) give the same bits, for daemons and walkers."""
    shape = (256, 12, 16, 1, 2)
    ref = None
    for xcd in (0, 1, 2):
        g = M.Lattice(*shape, seed=2026)
        g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_MULTISPIN)
        g.set_option(M.OPT_XCD_MAP, xcd)
        g.set_option(M.OPT_TILE_Y, 3)
        g.set_option(M.OPT_TILE_Z, 2)
        g.set_schedule(M.Schedule(M.SCHED_CONST, 0.8, 0.8, 60, 7))
        g.sweep(M.ALGO_MICSA, 15)
        g.sweep(M.ALGO_WALKERS, 11)
        got = (g.spins(), g.daemons(), g.energy_tally())
        if ref is None:
            ref = got
        else:
            assert all(np.array_equal(a, b) for a, b in zip(ref, got)), xcd
        g.close()


def test_multispin_refused_where_it_does_not_apply():
    g, _ = pair(96, 4, 4)
    with pytest.raises(M.MicsaError):
        g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_MULTISPIN)


def test_gpu_error_paths():
    g, _ = pair(8, 8, 8)
    with pytest.raises(M.MicsaError) as e:
        g.sweep(M.ALGO_MICSA, 1)
    assert e.value.status == M.ESTATE
    g.set_schedule(M.Schedule(M.SCHED_CONST, 1.0, 1.0, 5, 2))
    with pytest.raises(M.MicsaError) as e:
        g.sweep(M.ALGO_MICSA, 6)
    assert e.value.status == M.ERANGE
    with pytest.raises(M.MicsaError) as e:
        g.overlap(0, 0)
    assert e.value.status == M.EINVAL
    with pytest.raises(M.MicsaError) as e:
        g.write_daemons(np.full((1, 1, 512), 4, np.uint8))
    assert e.value.status == M.EINVAL
    with pytest.raises(M.MicsaError) as e:
        g.set_schedule(M.Schedule(M.SCHED_CONST, -1.0, 1.0, 5, 2))
    assert e.value.status == M.EINVAL
    with pytest.raises(M.MicsaError) as e:
        g.sweep(7, 1)
    assert e.value.status == M.EINVAL
    g.sweep(M.ALGO_MICSA, 5)
    assert g.counters() == (5, 2)


def test_timing_counts_launches():
    g, _ = pair(16, 16, 16)
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_SIMPLE)
    g.set_schedule(M.Schedule(M.SCHED_CONST, 1.5, 1.5, 20, 10))
    g.set_timing(True)
    g.sweep(M.ALGO_MICSA, 20)
    ms, n = g.timing(M.TIME_SWEEP)
    assert n == 40 and ms > 0  # two half-sweep launches per sweep
    ms_r, n_r = g.timing(M.TIME_REFRESH)
    assert n_r == 2
    h, _ = pair(16, 16, 16)
    h.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_RESIDENT)
    h.set_schedule(M.Schedule(M.SCHED_CONST, 1.5, 1.5, 20, 10))
    h.set_timing(True)
    h.sweep(M.ALGO_MICSA, 20)
    assert h.timing(M.TIME_SWEEP)[1] == 1  # all 20 sweeps in one launch
    m, _ = pair(16, 16, 16)
    m.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_SIMPLE)
    m.set_schedule(M.Schedule(M.SCHED_CONST, 1.5, 1.5, 20, 10))
    m.set_timing(True)
    m.sweep(M.ALGO_METROPOLIS, 7)
    assert m.timing(M.TIME_METROPOLIS)[1] == 14 and m.timing(M.TIME_HEATBATH)[1] == 0
    assert m.timing(M.TIME_SWEEP)[1] == 0


# ----------------------------------------------------------- fused sweep
FUSED_CASES = [
    ((32, 8, 8, 1, 1), 0, 0),
    ((32, 2, 2, 1, 2), 0, 0),     # minimum sides: ring rows/planes wrap onto the tile itself
    ((64, 6, 10, 2, 1), 0, 0),
    ((64, 6, 10, 2, 1), 1, 1),    # one-row, one-plane tiles
    ((32, 12, 4, 1, 2), 3, 2),
    ((96, 8, 6, 1, 1), 2, 3),     # three chunks per row
    ((128, 16, 16, 1, 1), 0, 0),
    ((64, 64, 64, 1, 2), 0, 0),   # the quench lattice
]


@pytest.mark.parametrize("algo", [M.ALGO_MICSA, M.ALGO_HEATBATH, M.ALGO_METROPOLIS])
@pytest.mark.parametrize("shape,ty,tz", FUSED_CASES)
def test_fused_sweep_matches_oracle(shape, ty, tz, algo):
    g, o = pair(*shape, seed=99)
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_FUSED)
    if ty:
        g.set_option(M.OPT_TILE_Y, ty)
    if tz:
        g.set_option(M.OPT_TILE_Z, tz)
    assert g.kernel_name(algo) in ("k_micsa_sweep_fused", "k_micsa_sweep2_fused", "k_heatbath_sweep_fused<0>",
                                   "k_heatbath_sweep_fused<1>")
    n = 23
    gs, os_ = scheds(M.SCHED_LINEAR, 2.5, 0.4, n, 5)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(algo, n, 1)
    Eo, Do = o.run(algo, os_, n, 1)
    assert np.array_equal(Eg, Eo)
    if algo == M.ALGO_MICSA:
        assert np.array_equal(Dg, Do)
    same_state(g, o)
    assert np.array_equal(g.energy_tally(), o.energy())


def test_every_launch_shape_gives_the_same_bits():
    """Launch shapes never change results: the fused sweep at every tile shape
    and the per-half kernels agree bit for bit (a racing or mis-indexed
    variant would not)."""
    shape = (64, 16, 12, 1, 2)
    n = 30
    ref = None
    variants = [(M.KERNEL_SIMPLE, 0, 0, 1, 1, 1), (M.KERNEL_RESIDENT, 0, 0, 1, 1, 1)] + [
        (M.KERNEL_FUSED, ty, tz, 1, pf, tp) for ty in (1, 2, 4, 8, 16) for tz in (1, 3, 4, 12) for pf in (1, 2)
        for tp in (1, 2)] + [(M.KERNEL_FUSED, 1, 3, 0, 1, 2), (M.KERNEL_FUSED, 4, 1, 0, 2, 1)]
    for kern, ty, tz, xcd, pf, tp in variants:
        g = M.Lattice(*shape, seed=2024)
        g.set_option(M.OPT_SWEEP_KERNEL, kern)
        g.set_option(M.OPT_XCD_MAP, xcd)
        g.set_option(M.OPT_PREFETCH, pf)
        g.set_option(M.OPT_TEMPORAL, tp)
        if ty:
            g.set_option(M.OPT_TILE_Y, ty)
            g.set_option(M.OPT_TILE_Z, tz)
        g.set_schedule(M.Schedule(M.SCHED_CONST, 0.8, 0.8, n, 7))
        E, D = g.sweep_logged(M.ALGO_MICSA, n, 5)  # odd stride: pairs and single sweeps, refreshes on either
        got = (E, D, g.spins(), g.daemons(), g.energy_tally())
        if ref is None:
            ref = got
        else:
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), (kern, ty, tz, xcd, pf, tp)
        g.close()


def test_tile_options_are_validated():
    g = M.Lattice(64, 12, 10, seed=1)
    for opt, v in ((M.OPT_TILE_Y, 13), (M.OPT_TILE_Z, 3), (M.OPT_SWEEP_KERNEL, 9)):
        with pytest.raises(M.MicsaError) as e:
            g.set_option(opt, v)
        assert e.value.status == M.EINVAL
    h = M.Lattice(40, 8, 8, seed=1)
    with pytest.raises(M.MicsaError) as e:
        h.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_FUSED)
    assert e.value.status == M.EINVAL
    big = M.Lattice(64, 64, 64, seed=1)  # 2.5 B/site does not fit one work-group's LDS
    with pytest.raises(M.MicsaError) as e:
        big.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_RESIDENT)
    assert e.value.status == M.EINVAL


# ------------------------------------------------------- bit-plane layout
def bpair(Lx, Ly, Lz, S, R, seed):
    return M.Lattice(Lx, Ly, Lz, S, R, seed, layout=M.LAYOUT_BITPLANE), O.Lattice(Lx, Ly, Lz, S, R, seed)


BIT_SHAPES = [
    (8, 4, 4, 1, 1),       # one live lane
    (8, 2, 2, 3, 2),       # minimum sides
    (16, 6, 10, 65, 2),    # two lane groups, the second with one live lane
    (24, 8, 6, 130, 1),    # three lane groups
    (32, 8, 8, 64, 3),
]


@pytest.mark.parametrize("shape", BIT_SHAPES)
def test_bitplane_trajectory_matches_oracle(shape):
    g, o = bpair(*shape, seed=31337)
    assert np.array_equal(g.couplings(), o.J)
    same_state(g, o)
    n = 25
    gs, os_ = scheds(M.SCHED_LINEAR, 2.2, 0.5, n, 6)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, n, 1)
    Eo, Do = o.run(O.ALGO_MICSA, os_, n, 1)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    same_state(g, o)
    if shape[4] > 1:
        assert np.array_equal(g.overlap(0, 1), o.overlap(0, 1))
    # the one-launch sweep keeps a per-lane incremental tally (conservation)
    assert g.kernel_name(M.ALGO_MICSA) == "kb_sweep"
    assert np.array_equal(g.energy_tally(), o.energy())


@pytest.mark.parametrize("shape,tz", [((16, 6, 10, 65, 2), 1), ((16, 6, 10, 65, 2), 2), ((8, 2, 2, 3, 2), 2),
                                      ((8, 2, 2, 3, 2), 1), ((32, 8, 8, 64, 3), 2), ((64, 32, 4, 70, 1), 1),
                                      ((64, 32, 4, 70, 1), 2)])
def test_bitplane_one_launch_tiles_match_oracle(shape, tz):
    """The one-launch bit-plane sweep with one and two planes per work-group
    (ring planes recomputed; planes that wrap onto a side of 2; two planes
    only where a plane has at most 512 words, else one), the largest plane of
    1024 words, two lane groups with a ragged last group."""
    g, o = bpair(*shape, seed=2718)
    g.set_option(M.OPT_TILE_Z, tz)
    n = 23
    gs, os_ = scheds(M.SCHED_LINEAR, 2.4, 0.3, n, 5)
    g.set_schedule(gs)
    for m in (9, 1, 13):
        g.sweep(M.ALGO_MICSA, m)
        o.run(O.ALGO_MICSA, os_, m, 0)
        same_state(g, o)
    assert g.kernel_name(M.ALGO_MICSA) == "kb_sweep"
    E = o.energy()
    assert np.array_equal(g.energy(), E) and np.array_equal(g.energy_tally(), E)
    assert np.array_equal(g.daemon_energy(), o.daemon_energy())


# planes of more than 1024 words: tiles of rows with two ring rows a side
ROW_TILE_SHAPES = [
    ((72, 30, 4, 65, 1), M.LANES_SAMPLES),    # 1080 words a plane: two tiles of 15 rows, two lane groups
    ((128, 18, 2, 3, 2), M.LANES_SAMPLES),    # 64 words a row, planes that wrap onto a side of 2
    ((64, 64, 6, 1, 20), M.LANES_REPLICAS),   # serving-size rows: tiles of 22, 22 and 20 rows
    ((64, 40, 4, 70, 1), M.LANES_SAMPLES),
]


@pytest.mark.parametrize("shape,lanes", ROW_TILE_SHAPES)
def test_bitplane_row_tiles_match_oracle(shape, lanes):
    """The one-launch bit-plane sweep on planes too large for one
    work-group (kb_sweep_rows, on request): refreshes every 4 sweeps, calls that split
    a refresh period, logged energies, per-lane tally and state against the
    oracle, in both lane modes."""
    Lx, Ly, Lz, S, R = shape
    g = M.Lattice(Lx, Ly, Lz, S, R, 0x7011, layout=M.LAYOUT_BITPLANE, lane_mode=lanes)
    o = O.Lattice(Lx, Ly, Lz, S, R, 0x7011)
    assert g.kernel_name(M.ALGO_MICSA) == "kb_micsa_half"  # the automatic choice on such planes
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_FUSED)
    assert g.kernel_name(M.ALGO_MICSA) == "kb_sweep_rows"
    gs, os_ = scheds(M.SCHED_LINEAR, 2.4, 0.3, 40, 4)
    g.set_schedule(gs)
    for m in (9, 1, 6):
        g.sweep(M.ALGO_MICSA, m)
        o.run(O.ALGO_MICSA, os_, m, 0)
        same_state(g, o)
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, 6, 2)
    Eo, Do = o.run(O.ALGO_MICSA, os_, 6, 2)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    same_state(g, o)
    E = o.energy()
    assert np.array_equal(g.energy(), E) and np.array_equal(g.energy_tally(), E)
    assert np.array_equal(g.daemon_energy(), o.daemon_energy())
    g.close()


def test_bitplane_batched_L32_shape():
    """256 samples x 2 replicas of L = 32 bit-packed in 4 lane groups, the
    launch the benchmark times (no option): 21 sweeps in one call (refreshes
    before sweeps 0, 10, 20), then 12 logged; per-lane tally equals the
    from-scratch energy of every lattice."""
    w = W.BATCHED_L32
    g, o = bpair(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
    gs, os_ = scheds(w.kind, w.T0, w.T1, w.n_sweeps, w.period)
    g.set_schedule(gs)
    g.sweep(M.ALGO_MICSA, 21)
    o.run(O.ALGO_MICSA, os_, 21, 0)
    same_state(g, o)
    assert np.array_equal(g.energy_tally(), o.energy())
    n = 12
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, n, 4)
    Eo, Do = o.run(O.ALGO_MICSA, os_, n, 4)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    assert np.array_equal(g.overlap(0, 1), o.overlap(0, 1))
    same_state(g, o)
    assert g.kernel_name(M.ALGO_MICSA) == "kb_sweep"
    assert np.array_equal(g.energy_tally(), o.energy())


@pytest.mark.parametrize("ahead", [0, 1], ids=["draw-in-place", "draw-ahead"])
def test_bitplane_long_calls_match_oracle(ahead):
    """Bit-plane layout, calls of many sweeps with a refresh every 3, the
    levels drawn just before each refresh sweep or ahead of it on the side
    stream while the sweeps before it run, against the oracle; two lane
    groups, two replicas."""
    g, o = bpair(32, 12, 10, 70, 2, seed=9090)
    g.set_option(M.OPT_DRAW_AHEAD, ahead)
    gs, os_ = scheds(M.SCHED_LINEAR, 2.5, 0.4, 80, 3)
    g.set_schedule(gs)
    for n in (31, 1, 2, 17):
        g.sweep(M.ALGO_MICSA, n)
        o.run(O.ALGO_MICSA, os_, n)
        same_state(g, o)
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, 12, 4)
    Eo, Do = o.run(O.ALGO_MICSA, os_, 12, 4)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    assert np.array_equal(g.overlap(0, 1), o.overlap(0, 1))


def test_layouts_are_bit_identical():
    """The same seed gives the same trajectory in the byte and bit-plane layouts."""
    shape = (32, 12, 10, 70, 2)
    n = 40
    res = []
    for layout in (M.LAYOUT_BYTE, M.LAYOUT_BITPLANE):
        g = M.Lattice(*shape, seed=4242, layout=layout)
        g.set_schedule(M.Schedule(M.SCHED_CONST, 0.8, 0.8, n, 10))
        E, D = g.sweep_logged(M.ALGO_MICSA, n, 5)
        res.append((E, D, g.spins(), g.daemons(), g.overlap(0, 1)))
        g.close()
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_bitplane_error_paths():
    g = M.Lattice(8, 4, 4, 3, 1, seed=1, layout=M.LAYOUT_BITPLANE)
    g.set_schedule(M.Schedule(M.SCHED_CONST, 1.0, 1.0, 10, 2))
    for algo in (M.ALGO_HEATBATH, M.ALGO_METROPOLIS, M.ALGO_WALKERS, 4):
        with pytest.raises(M.MicsaError) as e:
            g.sweep(algo, 1)
        assert e.value.status == M.EINVAL
    assert np.array_equal(g.energy_tally(), g.energy())
    # the per-half kernels keep no tally: it is refused until the spins are set again
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_SIMPLE)
    assert g.kernel_name(M.ALGO_MICSA) == "kb_micsa_half"
    g.sweep(M.ALGO_MICSA, 2)
    with pytest.raises(M.MicsaError) as e:
        g.energy_tally()
    assert e.value.status == M.ESTATE
    g.write_spins(g.spins())
    assert np.array_equal(g.energy_tally(), g.energy())
    # KERNEL_FUSED asks for the one-launch sweep; the byte-layout kernels are refused
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_FUSED)
    assert g.kernel_name(M.ALGO_MICSA) == "kb_sweep"
    for bad in (M.KERNEL_MULTISPIN, M.KERNEL_SLAB, M.KERNEL_RESIDENT):
        with pytest.raises(M.MicsaError) as e:
            g.set_option(M.OPT_SWEEP_KERNEL, bad)
        assert e.value.status == M.EINVAL


# ------------------------------------------------ gamma daemons / walkers
GAMMA_CASES = [
    ((16, 6, 10, 2, 2), 2, M.ALGO_MICSA),
    ((64, 8, 6, 1, 2), 4, M.ALGO_MICSA),
    ((8, 4, 4, 1, 3), 6, M.ALGO_WALKERS),
    ((32, 8, 8, 1, 1), 6, M.ALGO_WALKERS),
    ((24, 6, 4, 2, 1), 3, M.ALGO_WALKERS),
]


@pytest.mark.parametrize("shape,gamma,algo", GAMMA_CASES)
def test_gamma_trajectory_matches_oracle(shape, gamma, algo):
    """gamma daemons (walkers) per site: timesteps of gamma sweeps, family a on
    sweep a, refreshes at timestep boundaries, six wandering directions."""
    g = M.Lattice(*shape, seed=2024, gamma=gamma)
    o = O.Lattice(*shape, seed=2024, gamma=gamma)
    n = 9 * gamma + 2  # ends inside a timestep
    gs, os_ = scheds(M.SCHED_LINEAR, 2.4, 0.5, n + 5, 3)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(algo, n, 1)
    Eo, Do = o.run(algo, os_, n, 1)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    assert np.array_equal(g.spins(), o.sigma)
    assert g.daemons().shape == o.m.shape and np.array_equal(g.daemons(), o.m)
    assert np.array_equal(g.energy_tally(), o.energy())
    assert g.counters() == (n, (n // gamma) // 3)


def test_gamma_heatbath_uses_timestep_temperatures():
    g = M.Lattice(16, 4, 6, 1, 2, seed=31, gamma=3)
    o = O.Lattice(16, 4, 6, 1, 2, seed=31, gamma=3)
    gs, os_ = scheds(M.SCHED_LINEAR, 3.0, 0.3, 40, 2)
    g.set_schedule(gs)
    for algo in (M.ALGO_HEATBATH, M.ALGO_METROPOLIS):
        Eg, _ = g.sweep_logged(algo, 20, 1)
        Eo, _ = o.run(algo, os_, 20, 1)
        assert np.array_equal(Eg, Eo)
    assert np.array_equal(g.spins(), o.sigma)


def test_gamma_state_round_trip_and_options():
    g = M.Lattice(16, 4, 4, 2, 1, seed=3, gamma=4)
    m = np.random.default_rng(0).integers(0, 4, (2, 1, 4, g.N), dtype=np.uint8)
    g.write_daemons(m)
    assert np.array_equal(g.daemons(), m)
    D = g.daemon_energy()
    assert np.array_equal(D, 4 * m.reshape(2, -1).sum(axis=1).astype(np.int64))
    for kernel in (M.KERNEL_FUSED, M.KERNEL_RESIDENT):
        with pytest.raises(M.MicsaError) as e:
            g.set_option(M.OPT_SWEEP_KERNEL, kernel)
        assert e.value.status == M.EINVAL
    bad = m.copy()
    bad[0, 0, 3, 5] = 4
    with pytest.raises(M.MicsaError):
        g.write_daemons(bad)


# ------------------------------------------- C4 and coherence lengths (Sec. 3)
C4_CASES = [
    ((8, 4, 6, 1, 2), M.LAYOUT_BYTE),
    ((40, 10, 6, 2, 3), M.LAYOUT_BYTE),     # ragged rows (Kx = 20), three pairs
    ((64, 64, 64, 1, 2), M.LAYOUT_BYTE),    # the quench lattice
    ((96, 8, 4, 1, 4), M.LAYOUT_BYTE),      # Kx = 48: windows across words
    ((16, 8, 8, 70, 2), M.LAYOUT_BITPLANE), # two lane groups
]


@pytest.mark.parametrize("shape,layout", C4_CASES)
def test_c4_and_xi_match_oracle(shape, layout):
    g = M.Lattice(*shape, seed=808, layout=layout)
    o = O.Lattice(*shape, seed=808)
    n = 30
    gs, os_ = scheds(M.SCHED_CONST, 0.8, 0.8, n, 5)
    g.set_schedule(gs)
    g.sweep(M.ALGO_MICSA, n)
    o.run(O.ALGO_MICSA, os_, n, 0)
    assert np.array_equal(g.spins(), o.sigma)
    assert np.array_equal(g.c4_sums(), o.c4_sums())
    xg = g.xi()
    xo = o.xi()
    # same integer sums and the same double operations in the same order
    assert np.allclose(xg, xo, rtol=1e-13, atol=0, equal_nan=True), (xg, xo)
    assert np.array_equal(np.isnan(xg), np.isnan(xo))


def test_c4_needs_two_replicas():
    g = M.Lattice(8, 4, 4, 1, 1, seed=1)
    with pytest.raises(M.MicsaError) as e:
        g.c4_sums()
    assert e.value.status == M.EINVAL


def test_xi_of_written_overlap_fields_matches_oracle():
    """Finite coherence lengths: replica 1 is replica 0 with a slab and a
    checkerboard patch flipped, so C4 decays over a known range."""
    shape = (32, 16, 16, 2, 2)
    g = M.Lattice(*shape, seed=9)
    o = O.Lattice(*shape, seed=9)
    N = o.N
    i = np.arange(N)
    x, y, z = i % 32, (i // 32) % 16, i // 512
    flip = ((x < 8) | ((y < 4) & (z < 4))).astype(np.uint8)
    sig = o.sigma.copy()
    sig[:, 1] = sig[:, 0] ^ flip
    sig[1, 1] ^= ((x + y) % 5 == 0).astype(np.uint8)
    o.sigma[:] = sig
    g.write_spins(sig)
    assert np.array_equal(g.c4_sums(), o.c4_sums())
    xg, xo = g.xi(), o.xi()
    assert np.isfinite(xo).all()
    assert np.allclose(xg, xo, rtol=1e-13, atol=0), (xg, xo)


# ------------------------------------------------- two sweeps per pass
@pytest.mark.parametrize("shape,ty,tz", [((32, 2, 2, 1, 2), 0, 0), ((64, 6, 10, 2, 1), 1, 1), ((32, 12, 4, 1, 2), 3, 2),
                                         ((96, 8, 6, 1, 1), 2, 3), ((128, 16, 16, 1, 1), 0, 0),
                                         ((64, 64, 64, 1, 2), 0, 0), ((32, 4, 2, 1, 1), 4, 2)])
@pytest.mark.parametrize("period", [1, 2, 3])
def test_two_sweep_pass_matches_oracle(shape, ty, tz, period):
    """Sweeps k and k + 1 in one pass of the fused kernel: refreshes before the
    first, the second, both or neither sweep of a pair; minimum sides (rings
    that wrap several times onto the tile); ragged tiles."""
    g, o = pair(*shape, seed=31337)
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_FUSED)
    g.set_option(M.OPT_TEMPORAL, 2)
    if ty:
        g.set_option(M.OPT_TILE_Y, ty)
        g.set_option(M.OPT_TILE_Z, tz)
    assert g.kernel_name(M.ALGO_MICSA) == "k_micsa_sweep2_fused"
    n = 24
    gs, os_ = scheds(M.SCHED_LINEAR, 2.5, 0.4, n, period)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, n, 4)
    Eo, Do = o.run(O.ALGO_MICSA, os_, n, 4)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    same_state(g, o)
    assert np.array_equal(g.energy_tally(), o.energy())


def test_autotuner_gate_and_choice_match_oracle(tmp_path, monkeypatch):
    """The fused-sweep tuner on a small lattice: every candidate passes its
    bit-exact gate against the per-half kernel (tune raises otherwise), the
    cache is keyed and written, and the chosen launch shape reproduces the
    oracle's trajectory."""
    from paper_2506_16240_amd import tune

    monkeypatch.setattr(tune, "CACHE_PATH", str(tmp_path / "tune_cache.json"))
    shape = (128, 12, 8, 1, 2)
    best = tune.tune(*shape, sweeps=6, use_cache=True)
    assert (best.ty, best.tz) in tune.candidates(*shape[:3])
    assert best.us_per_sweep > 0
    again = tune.tune(*shape, sweeps=6, use_cache=True)  # from the cache
    assert again == best
    g, o = pair(*shape, seed=0x7E58)
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_FUSED)
    g.set_option(M.OPT_TILE_Y, best.ty)
    g.set_option(M.OPT_TILE_Z, best.tz)
    g.set_option(M.OPT_PREFETCH, best.prefetch)
    g.set_option(M.OPT_TEMPORAL, best.temporal)
    gs, os_ = scheds(M.SCHED_LINEAR, 2.5, 0.5, 30, 4)
    g.set_schedule(gs)
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, 30, 5)
    Eo, Do = o.run(O.ALGO_MICSA, os_, 30, 5)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    same_state(g, o)


# lanes = replicas of one sample, couplings broadcast (serving jobs of 1-64
# replicas of one instance; lane l of group g is replica 64 g + l)
REPLICA_SHAPES = [
    (16, 8, 8, 1, 5),     # one sample, five live lanes
    (8, 2, 2, 2, 3),      # minimum sides, two samples
    (32, 8, 6, 3, 70),    # two replica groups per sample
    (24, 6, 4, 1, 64),    # one full group
]


@pytest.mark.parametrize("shape", REPLICA_SHAPES)
def test_bitplane_replica_lanes_match_oracle(shape):
    Lx, Ly, Lz, S, R = shape
    g = M.Lattice(Lx, Ly, Lz, S, R, 0xBEEF, layout=M.LAYOUT_BITPLANE, lane_mode=M.LANES_REPLICAS)
    o = O.Lattice(Lx, Ly, Lz, S, R, 0xBEEF)
    assert np.array_equal(g.couplings(), o.J)
    same_state(g, o)
    n = 22
    gs, os_ = scheds(M.SCHED_LINEAR, 2.5, 0.4, n, 4)
    g.set_schedule(gs)
    g.sweep(M.ALGO_MICSA, 9)
    o.run(O.ALGO_MICSA, os_, 9, 0)
    same_state(g, o)
    Eg, Dg = g.sweep_logged(M.ALGO_MICSA, n - 9, 1)
    Eo, Do = o.run(O.ALGO_MICSA, os_, n - 9, 1)
    assert np.array_equal(Eg, Eo) and np.array_equal(Dg, Do)
    same_state(g, o)
    assert g.kernel_name(M.ALGO_MICSA) == "kb_sweep"
    assert np.array_equal(g.energy_tally(), o.energy())
    if R > 1:
        for a, b in ((0, R - 1), (1, 0), (0, min(R - 1, 65))):
            if a != b:
                assert np.array_equal(g.overlap(a, b), o.overlap(a, b))
        assert np.array_equal(g.c4_sums(), o.c4_sums())
    # the same lattices in the samples lane mode and in the byte layout agree
    for kw in (dict(layout=M.LAYOUT_BITPLANE), dict()):
        h = M.Lattice(Lx, Ly, Lz, S, R, 0xBEEF, **kw)
        h.set_schedule(gs)
        h.sweep(M.ALGO_MICSA, n)
        assert np.array_equal(h.spins(), o.sigma) and np.array_equal(h.daemons(), o.m)
        h.close()
    g.close()


def test_bitplane_replica_lanes_per_half_and_checkpoint():
    """The per-half kernels and a checkpoint split in the replicas lane mode."""
    shape = (16, 6, 4, 2, 7)
    gs, os_ = scheds(M.SCHED_CONST, 0.9, 0.9, 30, 5)
    o = O.Lattice(*shape, 99)
    o.run(O.ALGO_MICSA, os_, 30, 0)
    g = M.Lattice(*shape, 99, layout=M.LAYOUT_BITPLANE, lane_mode=M.LANES_REPLICAS)
    g.set_option(M.OPT_SWEEP_KERNEL, M.KERNEL_SIMPLE)
    g.set_schedule(gs)
    g.sweep(M.ALGO_MICSA, 12)
    image = g.save()
    g.close()
    h = M.Lattice(*shape, 99, layout=M.LAYOUT_BITPLANE, lane_mode=M.LANES_REPLICAS)
    h.load(image)
    h.sweep(M.ALGO_MICSA, 18)
    same_state(h, o)
    assert np.array_equal(h.energy_tally(), o.energy())
    # an image of one lane mode does not load into the other
    k = M.Lattice(*shape, 99, layout=M.LAYOUT_BITPLANE)
    assert M.lib().micsa_load(k._ctx, image, len(image)) == M.EINVAL
    k.close()
    h.close()
