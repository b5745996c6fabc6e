"""TEST INFRASTRUCTURE ONLY: Python face of the CPU oracle (oracle.c).

Only tests/, the smoke check and the benchmark's CPU-baseline leg use this
module.  The product library never imports it.  It wraps the plain C oracle
with ctypes and numpy and adds nothing to the arithmetic: every number
comes from oracle.c, which follows the paper (arXiv 2506.16240) step by step.

Arrays are in the oracle's natural order (site i = x + Lx*(y + Ly*z)):
  J[S, N]        bits 0..2 = forward-bond coupling bits j (J = 1 - 2j)
  sigma[S, R, N] spin bits (s = 1 - 2 sigma)
  m[S, R, N]     daemon levels (n = 4m); m[S, R, gamma, N] with gamma > 1
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MICSA_ORACLE_LIB points the tests at another build of oracle.c (the
# planted-mistake tests compile altered copies to check the pins fail).
LIB_PATH = os.environ.get("MICSA_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

ALGO_MICSA, ALGO_HEATBATH, ALGO_WALKERS, ALGO_METROPOLIS = 0, 1, 2, 3
SCHED_CONST, SCHED_LINEAR, SCHED_TABLE = 0, 1, 2
REFRESH_LOG2 = 0

_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
            "-Wall", "-Wextra", "-o", tmp, SRC_PATH, "-lm",
        ])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        c = ctypes
        L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.oracle_init_couplings.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64, _u8p]
        L.oracle_init_spins.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64, _u8p]
        L.oracle_daemon_thresholds.argtypes = [c.c_double, _u64p]
        L.oracle_heatbath_thresholds.argtypes = [c.c_double, _u64p]
        L.oracle_metropolis_thresholds.argtypes = [c.c_double, _u64p]
        L.oracle_refresh.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                     c.c_int64, c.c_double, _u8p]
        L.oracle_micsa_half.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int,
                                        c.c_int, _u8p, _u8p, _u8p, _i64p]
        L.oracle_micsa_site.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int64, _u8p, _u8p, _u8p]
        L.oracle_micsa_site.restype = c.c_int
        L.oracle_heatbath_half.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                           c.c_int64, c.c_int, c.c_double, _u8p, _u8p, _i64p]
        L.oracle_metropolis_half.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64,
                                             c.c_int64, c.c_int, c.c_double, _u8p, _u8p, _i64p]
        L.oracle_wander.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int,
                                    c.c_int, _u8p]
        L.oracle_energy.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, _u8p, _u8p, _i64p]
        L.oracle_daemon_energy.argtypes = [c.c_int64, c.c_int, _u8p, _i64p]
        L.oracle_overlap.argtypes = [c.c_int64, c.c_int, c.c_int, c.c_int, c.c_int, _u8p, _i64p]
        L.oracle_c4_sums.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, _u8p, c.c_int, _i64p]
        L.oracle_xi_from_c4.argtypes = [_f64p, c.c_int, c.POINTER(c.c_double), c.POINTER(c.c_double)]
        L.oracle_xi_from_c4.restype = c.c_int
        L.oracle_is_refresh.argtypes = [c.c_int64, c.c_int]
        L.oracle_is_refresh.restype = c.c_int
        L.oracle_refresh_index.argtypes = [c.c_int64, c.c_int]
        L.oracle_refresh_index.restype = c.c_int64
        L.oracle_refresh_count.argtypes = [c.c_int64, c.c_int]
        L.oracle_refresh_count.restype = c.c_int64
        L.oracle_temperature.argtypes = [c.c_int, c.c_double, c.c_double, c.c_int64, c.c_int,
                                         c.c_void_p, c.c_int64, c.c_int64]
        L.oracle_temperature.restype = c.c_double
        L.oracle_run.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64, c.c_int,
                                 c.c_int, c.c_double, c.c_double, c.c_int64, c.c_int, c.c_void_p,
                                 c.c_int64, c.c_int64, c.c_int64, c.c_int64, _u8p, _u8p, _u8p, _i64p,
                                 c.c_void_p, c.c_void_p]
        L.oracle_run.restype = c.c_int
        L.oracle_density_of_states.argtypes = [c.c_int, c.c_int, c.c_int, _u8p, _u64p]
        L.oracle_density_of_states.restype = c.c_int
        _i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        L.oracle_pt_quantise.argtypes = [c.c_int64, _f64p, _i32p]
        L.oracle_pt_quantise.restype = c.c_int
        L.oracle_pt_exp_table.argtypes = [c.c_double, _u64p]
        L.oracle_pt_exp_table.restype = c.c_int
        L.oracle_pt_exp_draw.argtypes = [_u64p, _u32p]
        L.oracle_pt_exp_draw.restype = c.c_int64
        L.oracle_pt_delta.argtypes = [c.c_int, c.c_int, c.c_int, _i32p, _u8p, c.c_int64]
        L.oracle_pt_delta.restype = c.c_int64
        L.oracle_pt_energy.argtypes = [c.c_int, c.c_int, c.c_int, _i32p, _u8p]
        L.oracle_pt_energy.restype = c.c_int64
        L.oracle_pt_init_spins.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint64, _u8p]
        L.oracle_pt_walker_refresh.argtypes = [c.c_int, c.c_int, c.c_int, c.c_uint64, c.c_int, c.c_int, c.c_int,
                                               c.c_int64, _u64p, _i64p]
        L.oracle_pt_creutz_half.argtypes = [c.c_int, c.c_int, c.c_int, _i32p, c.c_int, _u8p, _i64p]
        L.oracle_pt_creutz_half.restype = c.c_int64
        L.oracle_pt_wander_x.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, _i64p]
        L.oracle_pt_metropolis_half.argtypes = [c.c_int, c.c_int, c.c_int, _i32p, c.c_uint64, c.c_int, c.c_int,
                                                c.c_int, c.c_int64, c.c_int, _u64p, _u8p]
        L.oracle_pt_metropolis_half.restype = c.c_int64
        L.oracle_pt_houdayer.argtypes = [c.c_int, c.c_int, c.c_int, c.c_uint32, _u8p, _u8p]
        L.oracle_pt_houdayer.restype = c.c_int64
        L.oracle_pt_swap_step.argtypes = [c.c_int, c.c_int, c.c_int, _i32p, c.c_int, c.c_uint64, c.c_int, c.c_int,
                                          c.c_int64, _u64p, _u8p, c.c_void_p]
        L.oracle_pt_tables.argtypes = [c.c_int, _f64p, _u64p, _u64p]
        L.oracle_pt_tables.restype = c.c_int
        L.oracle_pt_run.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int,
                                    c.c_uint64, _i32p, _f64p, c.c_int64, c.c_int64, _u8p, c.c_void_p]
        L.oracle_pt_run.restype = c.c_int
        L.oracle_threads.restype = c.c_int
        L.oracle_set_threads.argtypes = [c.c_int]
        _lib = L
    return _lib


# ---------------------------------------------------------------- scalars
def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def daemon_thresholds(T: float) -> np.ndarray:
    t = np.zeros(3, np.uint64)
    lib().oracle_daemon_thresholds(float(T), t)
    return t


def heatbath_thresholds(T: float) -> np.ndarray:
    t = np.zeros(7, np.uint64)
    lib().oracle_heatbath_thresholds(float(T), t)
    return t


def metropolis_thresholds(T: float) -> np.ndarray:
    """theta[q], q = (dH + 12) / 4: a proposed flip with energy change dH is
    accepted iff the 32-bit uniform is below theta[q]."""
    t = np.zeros(7, np.uint64)
    lib().oracle_metropolis_thresholds(float(T), t)
    return t


def threads() -> int:
    return int(lib().oracle_threads())


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


@dataclass
class Schedule:
    """Temperature and refresh schedule (kind CONST / LINEAR / TABLE)."""
    kind: int = SCHED_CONST
    T0: float = 1.0
    T1: float = 1.0
    n_sweeps: int = 1
    period: int = 10          # >= 1: every `period` sweeps; 0: logarithmic
    table: np.ndarray | None = None

    def _table_args(self):
        if self.table is None:
            return None, 0
        t = np.ascontiguousarray(self.table, dtype=np.float64)
        return t, len(t)

    def temperature(self, rho: int, gamma: int = 1) -> float:
        """Temperature of refresh rho; with gamma sweeps per timestep the
        refreshes are counted over the timesteps that start in the schedule."""
        t, n = self._table_args()
        ptr = t.ctypes.data if t is not None else None
        n_steps = (self.n_sweeps + gamma - 1) // gamma
        return float(lib().oracle_temperature(self.kind, self.T0, self.T1, n_steps, self.period,
                                              ptr, n, int(rho)))

    def is_refresh(self, k: int) -> bool:
        return bool(lib().oracle_is_refresh(int(k), self.period))

    def refresh_index(self, k: int) -> int:
        return int(lib().oracle_refresh_index(int(k), self.period))

    def refresh_count(self, gamma: int = 1) -> int:
        return int(lib().oracle_refresh_count((self.n_sweeps + gamma - 1) // gamma, self.period))


@dataclass
class Lattice:
    """S samples x R replicas of an Lx x Ly x Lz periodic lattice, on the CPU,
    with gamma daemons (or walkers) per site."""
    Lx: int
    Ly: int
    Lz: int
    S: int = 1
    R: int = 1
    seed: int = 0
    gamma: int = 1
    J: np.ndarray = field(init=False)
    sigma: np.ndarray = field(init=False)
    m: np.ndarray = field(init=False)
    tally: np.ndarray = field(init=False)
    k: int = field(init=False, default=0)

    def __post_init__(self):
        for L in (self.Lx, self.Ly, self.Lz):
            if L < 2 or L % 2:
                raise ValueError("every side must be even and >= 2 (checkerboard, Sec. 2.1)")
        self.N = self.Lx * self.Ly * self.Lz
        self.J = np.zeros((self.S, self.N), np.uint8)
        self.sigma = np.zeros((self.S, self.R, self.N), np.uint8)
        if not 1 <= self.gamma <= 6:
            raise ValueError("gamma must be 1..6")
        self.m = np.zeros((self.S, self.R, self.N) if self.gamma == 1 else (self.S, self.R, self.gamma, self.N),
                          np.uint8)
        d = self._dims()
        lib().oracle_init_couplings(*d[:4], self.seed, self.J)
        lib().oracle_init_spins(*d, self.seed, self.sigma)
        self.tally = self.energy()

    def _dims(self):
        return (self.Lx, self.Ly, self.Lz, self.S, self.R)

    # -- single steps ---------------------------------------------------
    def refresh(self, rho: int, T: float) -> None:
        lib().oracle_refresh(*self._dims(), self.gamma, self.seed, int(rho), float(T), self.m)

    def micsa_half(self, parity: int, alpha: int = 0) -> None:
        """Half sweep with daemon family alpha."""
        if not 0 <= alpha < self.gamma:
            raise ValueError("alpha out of range")
        dE = np.zeros(self.S * self.R, np.int64)
        lib().oracle_micsa_half(*self._dims(), self.gamma, int(alpha), int(parity), self.J, self.sigma, self.m, dE)
        self.tally += dE

    def micsa_site(self, s: int, r: int, i: int) -> int:
        """One elementary move on site i of lattice (s, r) with its daemon of
        family 0; returns dH (0 if rejected)."""
        if self.gamma != 1:
            raise ValueError("micsa_site is for gamma = 1")
        sig = np.ascontiguousarray(self.sigma[s, r])
        m = np.ascontiguousarray(self.m[s, r])
        dH = int(lib().oracle_micsa_site(self.Lx, self.Ly, self.Lz, int(i), np.ascontiguousarray(self.J[s]),
                                         sig, m))
        self.sigma[s, r] = sig
        self.m[s, r] = m
        self.tally[s * self.R + r] += dH
        return dH

    def wander(self, direction: int, parity: int, alpha: int = 0) -> None:
        """Exchange walker `alpha` of every site of `parity` with that of its
        neighbour along `direction` (0..5 = +x, -x, +y, -y, +z, -z)."""
        if not 0 <= alpha < self.gamma:
            raise ValueError("alpha out of range")
        lib().oracle_wander(*self._dims(), self.gamma, int(alpha), int(direction), int(parity), self.m)

    def heatbath_half(self, k: int, parity: int, T: float) -> None:
        dE = np.zeros(self.S * self.R, np.int64)
        lib().oracle_heatbath_half(*self._dims(), self.seed, int(k), int(parity), float(T), self.J,
                                   self.sigma, dE)
        self.tally += dE

    def metropolis_half(self, k: int, parity: int, T: float) -> None:
        dE = np.zeros(self.S * self.R, np.int64)
        lib().oracle_metropolis_half(*self._dims(), self.seed, int(k), int(parity), float(T), self.J,
                                     self.sigma, dE)
        self.tally += dE

    # -- observables ----------------------------------------------------
    def energy(self) -> np.ndarray:
        E = np.zeros(self.S * self.R, np.int64)
        lib().oracle_energy(*self._dims(), self.J, self.sigma, E)
        return E

    def daemon_energy(self) -> np.ndarray:
        D = np.zeros(self.S * self.R, np.int64)
        lib().oracle_daemon_energy(self.N * self.gamma, self.S * self.R, self.m, D)
        return D

    def overlap(self, a: int, b: int) -> np.ndarray:
        Q = np.zeros(self.S, np.int64)
        lib().oracle_overlap(self.N, self.S, self.R, int(a), int(b), self.sigma, Q)
        return Q

    def c4_sums(self) -> np.ndarray:
        """G[S, 3, rmax+1]: sum over replica pairs a < b and sites of q_x q_{x+r e_mu}
        for r <= L_mu / 2 (0 beyond), rmax = max side / 2."""
        rmax = max(self.Lx, self.Ly, self.Lz) // 2
        G = np.zeros((self.S, 3, rmax + 1), np.int64)
        lib().oracle_c4_sums(*self._dims(), self.sigma, rmax, G)
        return G

    def c4(self) -> np.ndarray:
        """C4(r) [S, rmin+1], r = 0 .. min side / 2: mean over the three axes,
        normalised by N R (R-1) / 2."""
        G = self.c4_sums()
        rmin = min(self.Lx, self.Ly, self.Lz) // 2
        pairs = self.R * (self.R - 1) // 2
        return G[:, :, :rmin + 1].sum(axis=1) / (3.0 * self.N * pairs)

    def xi(self):
        """(xi12, xi23) per sample from C4 (eq. xi-def)."""
        out = []
        for row in self.c4():
            out.append(xi_from_c4(row))
        return np.array(out)

    # -- driver ---------------------------------------------------------
    def run(self, algo: int, sched: Schedule, n: int, stride: int = 0):
        """Sweeps k .. k+n-1; returns (E_log, D_log), each [n//stride, S*R]."""
        Lc = self.S * self.R
        rows = n // stride if stride > 0 else 0
        E_log = np.zeros((max(rows, 1), Lc), np.int64)
        D_log = np.zeros((max(rows, 1), Lc), np.int64)
        dE = np.zeros(Lc, np.int64)
        t, tn = sched._table_args()
        rc = lib().oracle_run(*self._dims(), self.gamma, self.seed, int(algo), sched.kind, sched.T0, sched.T1,
                              sched.n_sweeps, sched.period, t.ctypes.data if t is not None else None, tn,
                              self.k, int(n), int(stride), self.J, self.sigma, self.m, dE,
                              E_log.ctypes.data, D_log.ctypes.data)
        if rc != 0:
            raise ValueError("oracle_run rejected the schedule (non-positive or missing temperature)")
        self.tally += dE
        self.k += int(n)
        return E_log[:rows], D_log[:rows]


def xi_from_c4(C4) -> tuple[float, float]:
    """(xi12, xi23) from C4(r), r = 0..len-1 (eq. xi-def, integrals as sums);
    NaN when I1 or I2 is not positive (no correlation above the noise)."""
    c = np.ascontiguousarray(C4, np.float64)
    a, b = ctypes.c_double(), ctypes.c_double()
    if lib().oracle_xi_from_c4(c, len(c) - 1, ctypes.byref(a), ctypes.byref(b)) != 0:
        return float("nan"), float("nan")
    return a.value, b.value


def density_of_states(Lx: int, Ly: int, Lz: int, J: np.ndarray) -> np.ndarray:
    """Exact g(H) (uint64 counts, index (H + 3N)/2) of one sample by enumeration."""
    N = Lx * Ly * Lz
    g = np.zeros(3 * N + 1, np.uint64)
    rc = lib().oracle_density_of_states(Lx, Ly, Lz, np.ascontiguousarray(J, np.uint8), g)
    if rc != 0:
        raise ValueError("enumeration needs N <= 32")
    return g


def canonical_mean_energy(g: np.ndarray, N: int, T: float) -> float:
    """<H>_beta = sum_H H g(H) e^{-beta H} / sum_H g(H) e^{-beta H} (eq. canonical)."""
    H = -3 * N + 2 * np.arange(len(g), dtype=np.float64)
    beta = 1.0 / T
    w = g.astype(np.float64) * np.exp(-beta * (H - H.min()))
    return float((H * w).sum() / w.sum())


# ------------------------------------------------- App. C equilibrium workload
# Gaussian couplings on the energy mesh eps = 2^-17, continuous walkers
# (exponential on the mesh), parallel tempering with Houdayer moves; every
# number comes from the oracle_pt_* functions of oracle.c.
PT_WALKERS, PT_METROPOLIS = 0, 1
PT_MESH = 2.0 ** -17


def pt_quantise(J: np.ndarray) -> np.ndarray:
    """Couplings as integer multiples of the mesh (ValueError if |J| > 8 or not finite)."""
    J = np.ascontiguousarray(J, np.float64)
    Jq = np.zeros(J.shape, np.int32)
    if lib().oracle_pt_quantise(J.size, J.reshape(-1), Jq.reshape(-1)) != 0:
        raise ValueError("couplings must be finite with |J| <= 8")
    return Jq


def pt_exp_table(lam: float) -> tuple[np.ndarray, bool]:
    """[4, 255] digit thresholds of the mesh exponential of rate lam; ok is
    False if the top digit could reach 255."""
    t = np.zeros((4, 255), np.uint64)
    ok = lib().oracle_pt_exp_table(float(lam), t.reshape(-1)) == 0
    return t, ok


def pt_exp_draw(table: np.ndarray, w) -> int:
    return int(lib().oracle_pt_exp_draw(np.ascontiguousarray(table, np.uint64).reshape(-1),
                                        np.ascontiguousarray(w, np.uint32)))


def pt_tables(T) -> tuple[np.ndarray, np.ndarray]:
    """Walker tables [M, 4, 255] (rate beta_t) and pair tables [M-1, 4, 255]
    (rate beta_t - beta_{t+1}); ValueError for an invalid ladder."""
    T = np.ascontiguousarray(T, np.float64)
    M = len(T)
    wt = np.zeros((M, 4, 255), np.uint64)
    pt = np.zeros((max(M - 1, 1), 4, 255), np.uint64)
    if lib().oracle_pt_tables(M, T, wt.reshape(-1), pt.reshape(-1)) != 0:
        raise ValueError("temperatures must be positive and strictly increasing, within the sampler's range")
    return wt, pt[:M - 1]


def pt_delta(dims, Jq, sig, i: int) -> int:
    return int(lib().oracle_pt_delta(*dims, Jq.reshape(-1), sig, int(i)))


def pt_energy(dims, Jq, sig) -> int:
    return int(lib().oracle_pt_energy(*dims, Jq.reshape(-1), sig))


def pt_walker_refresh(dims, seed, run, rep, t, e, table) -> np.ndarray:
    n = np.zeros(dims[0] * dims[1] * dims[2], np.int64)
    lib().oracle_pt_walker_refresh(*dims, seed, run, rep, t, e, np.ascontiguousarray(table).reshape(-1), n)
    return n


def pt_creutz_half(dims, Jq, parity, sig, n) -> int:
    return int(lib().oracle_pt_creutz_half(*dims, Jq.reshape(-1), parity, sig, n))


def pt_wander_x(dims, parity, n) -> None:
    lib().oracle_pt_wander_x(*dims, parity, n)


def pt_metropolis_half(dims, Jq, seed, run, rep, t, k, parity, table, sig) -> int:
    return int(lib().oracle_pt_metropolis_half(*dims, Jq.reshape(-1), seed, run, rep, t, k, parity,
                                               np.ascontiguousarray(table).reshape(-1), sig))


def pt_houdayer(dims, u: int, sa, sb) -> int:
    return int(lib().oracle_pt_houdayer(*dims, int(u) & 0xFFFFFFFF, sa, sb))


def pt_swap_step(dims, Jq, seed, run, rep, e, pair_tables, sig, swaps=None) -> None:
    """sig[M, N]: the configurations of one replica group by temperature."""
    M = sig.shape[0]
    lib().oracle_pt_swap_step(*dims, Jq.reshape(-1), M, seed, run, rep, e,
                              np.ascontiguousarray(pair_tables, np.uint64).reshape(-1), sig.reshape(-1),
                              None if swaps is None else swaps.ctypes.data)


@dataclass
class PTLattice:
    """runs x 2 replicas x M temperatures of one Gaussian sample J[3, N]."""
    Lx: int
    Ly: int
    Lz: int
    runs: int
    T: np.ndarray
    J: np.ndarray
    seed: int
    sweeps: int = 10
    algo: int = PT_WALKERS
    houdayer: bool = True
    e: int = 0
    sigma: np.ndarray = field(default=None, repr=False)   # [runs, 2, M, N] by temperature

    def __post_init__(self):
        self.T = np.ascontiguousarray(self.T, np.float64)
        self.M = len(self.T)
        self.N = self.Lx * self.Ly * self.Lz
        self.Jq = pt_quantise(np.asarray(self.J, np.float64).reshape(3, self.N))
        if self.sigma is None:
            self.sigma = np.zeros((self.runs, 2, self.M, self.N), np.uint8)
            lib().oracle_pt_init_spins(self.Lx, self.Ly, self.Lz, self.runs, self.M, self.seed,
                                       self.sigma.reshape(-1))

    @property
    def dims(self):
        return (self.Lx, self.Ly, self.Lz)

    def run(self, n_emcs: int, swaps: np.ndarray | None = None) -> None:
        st = lib().oracle_pt_run(self.Lx, self.Ly, self.Lz, self.runs, self.M, self.sweeps, self.algo,
                                 int(self.houdayer), self.seed, self.Jq.reshape(-1), self.T, self.e, n_emcs,
                                 self.sigma.reshape(-1), None if swaps is None else swaps.ctypes.data)
        if st != 0:
            raise ValueError("invalid temperature ladder")
        self.e += n_emcs

    def energies(self) -> np.ndarray:
        """[runs, 2, M] H in units of the mesh."""
        E = np.zeros((self.runs, 2, self.M), np.int64)
        for u in range(self.runs):
            for r in range(2):
                for t in range(self.M):
                    E[u, r, t] = pt_energy(self.dims, self.Jq, self.sigma[u, r, t])
        return E

    def overlaps(self) -> np.ndarray:
        """[runs, M] Q = sum_x s^a_x s^b_x of the two replicas at each temperature."""
        s = 1 - 2 * self.sigma.astype(np.int64)
        return (s[:, 0] * s[:, 1]).sum(axis=-1)
