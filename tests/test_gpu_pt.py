"""GPU parity of the equilibrium workload (App. C): parallel tempering of a
Gaussian sample with continuous walkers (or Metropolis) and Houdayer moves,
through the C ABI, against the CPU oracle.

All arithmetic is integer on the 2^-17 energy mesh and every random number
has a fixed counter, so the trajectory is unique: parity is bit equality of
the spins by temperature, the energies, the overlaps and the exchange counts.
Shapes cover the smallest sides, x rows of 2 and 64 sites, ragged y/z, the
paper's L = 10 with its 40 temperatures, coupling records read from global
memory (large N), and the full 200-run workload for one EMCS.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_16240_amd import micsa as M
from paper_2506_16240_amd import workloads as W

pytestmark = pytest.mark.gpu


def make(dims, runs, T, seed, sweeps=10, algo=M.PT_WALKERS, houdayer=True, jseed=None, kernel=M.PT_KERNEL_AUTO):
    J = W.gaussian_couplings(*dims, seed if jseed is None else jseed)
    g = M.PT(*dims, runs, T, J, seed, sweeps, algo, houdayer)
    g.set_kernel(kernel)
    o = O.PTLattice(*dims, runs=runs, T=T, J=J, seed=seed, sweeps=sweeps,
                    algo=O.PT_WALKERS if algo == M.PT_WALKERS else O.PT_METROPOLIS, houdayer=houdayer)
    return g, o


def same(g, o, swaps=None):
    assert np.array_equal(g.spins(), o.sigma), "spins differ"
    E, Q = g.read()
    assert np.array_equal(E, o.energies()), "energies differ"
    assert np.array_equal(Q, o.overlaps()), "overlaps differ"
    if swaps is not None:
        assert np.array_equal(g.swaps(), swaps), "exchange counts differ"


def test_tables_and_couplings_match_oracle():
    T = np.linspace(0.2, 2.0, 40)
    g, o = make((10, 10, 10), 1, T, 3)
    assert np.array_equal(g.couplings(), o.Jq)
    wt, pt = O.pt_tables(T)
    for t in range(40):
        assert np.array_equal(g.tables(0, t), wt[t])
    for t in range(39):
        assert np.array_equal(g.tables(1, t), pt[t])
    same(g, o)
    g.close()


CASES = [
    # dims, runs, T, sweeps, algo, houdayer, n_emcs
    ((2, 2, 2), 3, [0.5, 1.0, 2.0], 10, M.PT_WALKERS, True, 12),
    ((4, 4, 4), 3, [0.4, 0.9], 10, M.PT_WALKERS, True, 10),
    ((6, 4, 8), 2, [0.3, 0.5, 0.8, 1.2, 2.0], 3, M.PT_WALKERS, True, 8),
    ((64, 4, 2), 2, [0.3, 0.6, 1.5], 5, M.PT_WALKERS, True, 6),
    ((8, 6, 10), 2, [0.3, 0.5, 0.8, 1.2, 2.0], 10, M.PT_WALKERS, False, 6),
    ((4, 4, 4), 3, [0.4, 0.9], 10, M.PT_METROPOLIS, True, 10),
    ((6, 4, 8), 2, [0.3, 0.5, 0.8, 1.2, 2.0], 3, M.PT_METROPOLIS, True, 6),
    ((64, 4, 2), 2, [0.3, 0.6, 1.5], 4, M.PT_METROPOLIS, False, 4),
    ((10, 10, 10), 2, list(np.linspace(0.2, 2.0, 40)), 10, M.PT_WALKERS, True, 6),
    ((10, 10, 10), 2, list(np.linspace(0.2, 2.0, 40)), 10, M.PT_METROPOLIS, True, 3),
]


REGISTER_LX = (4, 6, 8, 10, 12, 16)


@pytest.mark.parametrize("kernel", [M.PT_KERNEL_AUTO, M.PT_KERNEL_ROWS], ids=["auto", "rows"])
@pytest.mark.parametrize("dims,runs,T,sweeps,algo,houdayer,n", CASES,
                         ids=[f"{c[0][0]}x{c[0][1]}x{c[0][2]}-r{c[1]}-M{len(c[2])}-s{c[3]}-a{c[4]}-h{int(c[5])}"
                              for c in CASES])
def test_trajectory_matches_oracle(dims, runs, T, sweeps, algo, houdayer, n, kernel):
    g, o = make(dims, runs, np.array(T), 0x5EED0100 + runs * 7 + sweeps, sweeps, algo, houdayer, kernel=kernel)
    reg = kernel == M.PT_KERNEL_AUTO and dims[0] in REGISTER_LX and 2 * dims[1] * dims[2] <= 1024
    assert g.kernel_name == ("k_pt_emcs_reg" if reg else "k_pt_emcs")
    same(g, o)
    swaps = np.zeros((runs, 2, len(T) - 1), np.int64)
    for chunk in (1, n - 1):  # one EMCS, then the rest in one call
        g.step(chunk)
        o.run(chunk, swaps)
        same(g, o, swaps)
    assert g.emcs == n
    g.close()


@pytest.mark.parametrize("kernel", [M.PT_KERNEL_AUTO, M.PT_KERNEL_ROWS], ids=["register", "rows"])
def test_large_lattice(kernel):
    """16^3 sites: the register kernel holds one temperature per work-group;
    the row kernel has no room for the coupling records in LDS and reads
    them from global memory."""
    g, o = make((16, 16, 16), 1, np.array([0.5, 1.0, 1.5]), 0x5EED0200, sweeps=4, kernel=kernel)
    assert g.kernel_name == ("k_pt_emcs_reg" if kernel == M.PT_KERNEL_AUTO else "k_pt_emcs")
    swaps = np.zeros((1, 2, 2), np.int64)
    g.step(3)
    o.run(3, swaps)
    same(g, o, swaps)
    g.close()


def test_register_kernel_refused_where_it_does_not_apply():
    g, _ = make((64, 4, 2), 1, np.array([0.5, 1.0]), 9)
    with pytest.raises(M.MicsaError):
        g.set_kernel(M.PT_KERNEL_REGISTER)
    assert g.kernel_name == "k_pt_emcs"
    g.close()


def test_injected_states():
    """Equal replicas (no Houdayer cluster), opposite replicas (one cluster
    of every site) and a low-temperature ladder from written states."""
    dims, runs, T = (6, 6, 6), 2, np.array([0.2, 0.25, 0.3])
    g, o = make(dims, runs, T, 0x5EED0300, sweeps=2)
    rng = np.random.default_rng(5)
    sig = rng.integers(0, 2, (runs, 2, 3, 216)).astype(np.uint8)
    sig[0, 1] = sig[0, 0]          # run 0: replicas equal
    sig[1, 1] = sig[1, 0] ^ 1      # run 1: replicas opposite
    g.write_spins(sig)
    o.sigma[...] = sig
    same(g, o)
    swaps = np.zeros((runs, 2, 2), np.int64)
    g.step(4)
    o.run(4, swaps)
    same(g, o, swaps)
    g.close()


@pytest.mark.parametrize("algo", [M.PT_WALKERS, M.PT_METROPOLIS])
def test_full_workload_first_emcs(algo):
    """The paper's set-up at full size (L = 10, 200 runs, 40 temperatures,
    10 sweeps per EMCS) in the launch configuration the benchmark times:
    every run, temperature and replica after the first EMCS."""
    w = W.PT_L10
    T = w.temperatures()
    g = M.PT(w.L, w.L, w.L, w.runs, T, w.couplings(), w.seed, w.sweeps, algo, True)
    assert g.kernel_name == "k_pt_emcs_reg"
    o = O.PTLattice(w.L, w.L, w.L, runs=w.runs, T=T, J=w.couplings(), seed=w.seed, sweeps=w.sweeps,
                    algo=O.PT_WALKERS if algo == M.PT_WALKERS else O.PT_METROPOLIS, houdayer=True)
    swaps = np.zeros((w.runs, 2, w.M - 1), np.int64)
    g.step(1)
    o.run(1, swaps)
    same(g, o, swaps)
    g.close()


def test_timing_and_range():
    g, _ = make((4, 4, 4), 1, np.array([0.5, 1.0]), 7)
    g.set_timing(True)
    g.step(3)
    ms0, n0 = g.timing(M.PT_TIME_EMCS)
    ms1, n1 = g.timing(M.PT_TIME_SWAP)
    assert n0 == 3 and n1 == 3 and ms0 > 0 and ms1 > 0
    with pytest.raises(M.MicsaError):
        g.step(1 << 32)
    assert g.emcs == 3
    g.close()
