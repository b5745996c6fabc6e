"""Python binding of libmicsa (include/micsa.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts
numpy arrays and Python values to the C ABI and raises on error statuses.
If libmicsa.so has not been built the import of the library fails loudly:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmicsa.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, ERANGE = 0, -1, -2, -3, -4, -5
LAYOUT_BYTE, LAYOUT_BITPLANE = 0, 1
LANES_SAMPLES, LANES_REPLICAS = 0, 1
ALGO_MICSA, ALGO_HEATBATH, ALGO_WALKERS, ALGO_METROPOLIS = 0, 1, 2, 3
SCHED_CONST, SCHED_LINEAR, SCHED_TABLE = 0, 1, 2
REFRESH_LOG2 = 0
TIME_SWEEP, TIME_REFRESH, TIME_HEATBATH, TIME_REDUCE, TIME_METROPOLIS = 0, 1, 2, 3, 4
OPT_SWEEP_KERNEL, OPT_TILE_Y, OPT_TILE_Z, OPT_XCD_MAP, OPT_GRAPHS, OPT_PREFETCH, OPT_TEMPORAL, OPT_MSC_FUSED = 1, 2, 3, 4, 5, 6, 7, 8
OPT_DRAW_AHEAD = 9
OPT_MSC_PASS = 10
KERNEL_AUTO, KERNEL_SIMPLE, KERNEL_FUSED, KERNEL_RESIDENT, KERNEL_MULTISPIN, KERNEL_SLAB = 0, 1, 2, 3, 4, 5
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_RELEASED = 0, 1, 2, 3
PT_WALKERS, PT_METROPOLIS = 0, 1
PT_TIME_EMCS, PT_TIME_SWAP = 0, 1
PT_KERNEL_AUTO, PT_KERNEL_ROWS, PT_KERNEL_REGISTER = 0, 1, 2
PT_MAX_SITES = 16384


class MicsaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("Lz", ctypes.c_int32),
                ("n_samples", ctypes.c_int32), ("n_replicas", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("gamma", ctypes.c_int32), ("lane_mode", ctypes.c_int32), ("seed", ctypes.c_uint64)]


def _params(Lx, Ly, Lz, S, R, layout, seed, gamma=1, lane_mode=0) -> _Params:
    return _Params(Lx=Lx, Ly=Ly, Lz=Lz, n_samples=S, n_replicas=R, layout=layout, gamma=gamma,
                   lane_mode=lane_mode, seed=seed & (2**64 - 1))


class _Schedule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("refresh_period", ctypes.c_int32), ("T0", ctypes.c_double),
                ("T1", ctypes.c_double), ("n_sweeps", ctypes.c_int64),
                ("T_table", ctypes.POINTER(ctypes.c_double)), ("T_len", ctypes.c_int64)]


_lib = None

class _PtParams(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("Lz", ctypes.c_int32),
                ("n_runs", ctypes.c_int32), ("n_temps", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("algo", ctypes.c_int32), ("houdayer", ctypes.c_int32), ("seed", ctypes.c_uint64)]


# (name, restype, argtypes) of every exported entry point
_SIGNATURES = [
    ("micsa_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("micsa_last_error", ctypes.c_char_p, [ctypes.c_void_p]),
    ("micsa_create", ctypes.c_int, [ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    ("micsa_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("micsa_set_schedule", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Schedule)]),
    ("micsa_sweep", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64]),
    ("micsa_sweep_logged", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_sweep_logged_d", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_sync", ctypes.c_int, [ctypes.c_void_p]),
    ("micsa_read_energy", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_read_energy_tally", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_read_demon_energy", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_read_overlap", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    ("micsa_read_spins", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_read_demons", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_read_couplings", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_get_counters", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int64)]),
    ("micsa_get_thresholds", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    ("micsa_get_heatbath_thresholds", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    ("micsa_get_metropolis_thresholds", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    ("micsa_read_c4", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_read_c4_static", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_read_xi", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_write_spins", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_write_demons", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_save", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    ("micsa_load", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    ("micsa_set_timing", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("micsa_get_timing", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64)]),
    ("micsa_kernel_name", ctypes.c_char_p, [ctypes.c_void_p, ctypes.c_int32]),
    ("micsa_set_option", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64]),
    ("micsa_pool_footprint", ctypes.c_int, [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_size_t)]),
    ("micsa_pool_create", ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    ("micsa_pool_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("micsa_pool_submit", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Params), ctypes.POINTER(_Schedule),
                                         ctypes.POINTER(ctypes.c_int64)]),
    ("micsa_pool_step", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    ("micsa_pool_sync", ctypes.c_int, [ctypes.c_void_p]),
    ("micsa_pool_job_state", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int64)]),
    ("micsa_pool_job_context", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p)]),
    ("micsa_pool_release", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    ("micsa_pt_create", ctypes.c_int, [ctypes.POINTER(_PtParams), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_void_p)]),
    ("micsa_pt_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("micsa_pt_last_error", ctypes.c_char_p, [ctypes.c_void_p]),
    ("micsa_pt_step", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    ("micsa_pt_sync", ctypes.c_int, [ctypes.c_void_p]),
    ("micsa_pt_get_emcs", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    ("micsa_pt_read", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_pt_read_spins", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_pt_write_spins", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_pt_read_swaps", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_pt_get_tables", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    ("micsa_pt_get_couplings", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("micsa_pt_set_kernel", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("micsa_pt_kernel_name", ctypes.c_char_p, [ctypes.c_void_p]),
    ("micsa_pt_set_timing", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("micsa_pt_get_timing", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64)]),
]


def exported_symbols() -> list[str]:
    return [s[0] for s in _SIGNATURES]


def lib():
    """Load libmicsa.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def _stream_handle(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


@dataclass
class Schedule:
    kind: int = SCHED_CONST
    T0: float = 1.0
    T1: float = 1.0
    n_sweeps: int = 1
    period: int = 10
    table: np.ndarray | None = None


def _schedule_struct(s: "Schedule"):
    tab, n, keep = None, 0, None
    if s.table is not None:
        keep = np.ascontiguousarray(s.table, np.float64)
        tab, n = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(keep)
    return _Schedule(s.kind, s.period, s.T0, s.T1, s.n_sweeps, tab, n), keep


class Lattice:
    """S samples x R replicas on the GPU (one libmicsa context)."""

    _owned = True

    @classmethod
    def _borrow(cls, ctx: ctypes.c_void_p, Lx, Ly, Lz, S, R, seed=0, gamma=1) -> "Lattice":
        """A view of a context owned by someone else (a pool job): never destroyed here."""
        obj = cls.__new__(cls)
        obj.Lx, obj.Ly, obj.Lz, obj.S, obj.R = Lx, Ly, Lz, S, R
        obj.N = Lx * Ly * Lz
        obj.seed = seed
        obj.gamma = gamma
        obj._ctx = ctx
        obj._owned = False
        obj._table = None
        return obj

    def __init__(self, Lx: int, Ly: int, Lz: int, S: int = 1, R: int = 1, seed: int = 0,
                 layout: int = LAYOUT_BYTE, stream=None, gamma: int = 1, lane_mode: int = LANES_SAMPLES):
        self.Lx, self.Ly, self.Lz, self.S, self.R = Lx, Ly, Lz, S, R
        self.N = Lx * Ly * Lz
        self.seed = seed
        self.gamma = gamma
        self._ctx = ctypes.c_void_p()
        p = _params(Lx, Ly, Lz, S, R, layout, seed, gamma, lane_mode)
        st = lib().micsa_create(ctypes.byref(p), _stream_handle(stream), ctypes.byref(self._ctx))
        if st != OK:
            raise MicsaError(st, f"micsa_create({Lx},{Ly},{Lz},S={S},R={R}): "
                                 f"{lib().micsa_status_string(st).decode()}")
        self._table = None

    # -- plumbing -------------------------------------------------------
    def _check(self, st: int, what: str) -> None:
        if st != OK:
            msg = lib().micsa_last_error(self._ctx).decode()
            raise MicsaError(st, f"{what}: {lib().micsa_status_string(st).decode()}: {msg}")

    def close(self) -> None:
        if self._ctx and self._owned:
            lib().micsa_destroy(self._ctx)
        self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- schedule and sweeps --------------------------------------------
    def set_schedule(self, s: Schedule) -> None:
        cs, self._table = _schedule_struct(s)
        self._check(lib().micsa_set_schedule(self._ctx, ctypes.byref(cs)), "set_schedule")

    def sweep(self, algo: int, n: int) -> None:
        self._check(lib().micsa_sweep(self._ctx, algo, n), "sweep")

    def sweep_logged(self, algo: int, n: int, stride: int = 1):
        rows = n // stride
        E = np.zeros((rows, self.S * self.R), np.int64)
        D = np.zeros((rows, self.S * self.R), np.int64)
        self._check(lib().micsa_sweep_logged(self._ctx, algo, n, stride, _ptr(E), _ptr(D)), "sweep_logged")
        return E, D

    def sweep_logged_d(self, algo: int, n: int, stride: int, E_log, D_log) -> None:
        """micsa_sweep_logged_d: E_log / D_log are device int64 buffers of
        [n // stride][S * R] entries (objects with data_ptr(), raw addresses
        or None); enqueue only."""
        def addr(t):
            return None if t is None else (t.data_ptr() if hasattr(t, "data_ptr") else int(t))
        self._check(lib().micsa_sweep_logged_d(self._ctx, algo, n, stride, addr(E_log), addr(D_log)),
                    "sweep_logged_d")

    def sync(self) -> None:
        self._check(lib().micsa_sync(self._ctx), "sync")

    def save(self) -> bytes:
        """Checkpoint image (micsa_save)."""
        n = ctypes.c_size_t(0)
        self._check(lib().micsa_save(self._ctx, None, ctypes.byref(n)), "save (size)")
        buf = ctypes.create_string_buffer(n.value)
        self._check(lib().micsa_save(self._ctx, buf, ctypes.byref(n)), "save")
        return buf.raw[:n.value]

    def load(self, image: bytes) -> None:
        """Restore a checkpoint image (micsa_load)."""
        self._check(lib().micsa_load(self._ctx, image, len(image)), "load")


    # -- reads ----------------------------------------------------------
    def _read_vec(self, fn, n, what):
        out = np.zeros(n, np.int64)
        self._check(fn(self._ctx, _ptr(out)), what)
        return out

    def energy(self) -> np.ndarray:
        return self._read_vec(lib().micsa_read_energy, self.S * self.R, "read_energy")

    def energy_tally(self) -> np.ndarray:
        return self._read_vec(lib().micsa_read_energy_tally, self.S * self.R, "read_energy_tally")

    def daemon_energy(self) -> np.ndarray:
        return self._read_vec(lib().micsa_read_demon_energy, self.S * self.R, "read_demon_energy")

    def overlap(self, a: int, b: int) -> np.ndarray:
        out = np.zeros(self.S, np.int64)
        self._check(lib().micsa_read_overlap(self._ctx, a, b, _ptr(out)), "read_overlap")
        return out

    def spins(self) -> np.ndarray:
        out = np.zeros((self.S, self.R, self.N), np.uint8)
        self._check(lib().micsa_read_spins(self._ctx, _ptr(out)), "read_spins")
        return out

    def _daemon_shape(self):
        return (self.S, self.R, self.N) if self.gamma == 1 else (self.S, self.R, self.gamma, self.N)

    def c4_sums(self) -> np.ndarray:
        """G[S, 3, rmax+1] (micsa_read_c4), rmax = max side / 2."""
        rmax = max(self.Lx, self.Ly, self.Lz) // 2
        out = np.zeros((self.S, 3, rmax + 1), np.int64)
        self._check(lib().micsa_read_c4(self._ctx, _ptr(out)), "read_c4")
        return out

    def c4_sums_static(self) -> np.ndarray:
        """As c4_sums, through micsa_read_c4_static (no device allocation)."""
        rmax = max(self.Lx, self.Ly, self.Lz) // 2
        out = np.zeros((self.S, 3, rmax + 1), np.int64)
        self._check(lib().micsa_read_c4_static(self._ctx, _ptr(out)), "read_c4_static")
        return out

    def xi(self) -> np.ndarray:
        """[S, 2]: (xi12, xi23) per sample (micsa_read_xi)."""
        a = np.zeros(self.S, np.float64)
        b = np.zeros(self.S, np.float64)
        self._check(lib().micsa_read_xi(self._ctx, _ptr(a), _ptr(b)), "read_xi")
        return np.stack([a, b], axis=1)

    def daemons(self) -> np.ndarray:
        """Levels [S, R, N] (gamma = 1) or [S, R, gamma, N]."""
        out = np.zeros(self._daemon_shape(), np.uint8)
        self._check(lib().micsa_read_demons(self._ctx, _ptr(out)), "read_demons")
        return out

    def couplings(self) -> np.ndarray:
        out = np.zeros((self.S, self.N), np.uint8)
        self._check(lib().micsa_read_couplings(self._ctx, _ptr(out)), "read_couplings")
        return out

    def counters(self) -> tuple[int, int]:
        k, rho = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().micsa_get_counters(self._ctx, ctypes.byref(k), ctypes.byref(rho)), "get_counters")
        return k.value, rho.value

    def thresholds(self, rho: int) -> np.ndarray:
        t = np.zeros(3, np.uint64)
        self._check(lib().micsa_get_thresholds(self._ctx, rho, _ptr(t)), "get_thresholds")
        return t

    def heatbath_thresholds(self, rho: int) -> np.ndarray:
        t = np.zeros(7, np.uint64)
        self._check(lib().micsa_get_heatbath_thresholds(self._ctx, rho, _ptr(t)), "get_heatbath_thresholds")
        return t

    def metropolis_thresholds(self, rho: int) -> np.ndarray:
        t = np.zeros(7, np.uint64)
        self._check(lib().micsa_get_metropolis_thresholds(self._ctx, rho, _ptr(t)), "get_metropolis_thresholds")
        return t

    # -- writes ---------------------------------------------------------
    def write_spins(self, sigma: np.ndarray) -> None:
        a = np.ascontiguousarray(sigma, np.uint8).reshape(self.S, self.R, self.N)
        self._check(lib().micsa_write_spins(self._ctx, _ptr(a)), "write_spins")

    def write_daemons(self, m: np.ndarray) -> None:
        a = np.ascontiguousarray(m, np.uint8).reshape(self._daemon_shape())
        self._check(lib().micsa_write_demons(self._ctx, _ptr(a)), "write_demons")

    # -- timing ---------------------------------------------------------
    def set_timing(self, enable: bool) -> None:
        self._check(lib().micsa_set_timing(self._ctx, 1 if enable else 0), "set_timing")

    def timing(self, kind: int) -> tuple[float, int]:
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(lib().micsa_get_timing(self._ctx, kind, ctypes.byref(ms), ctypes.byref(n)), "get_timing")
        return ms.value, n.value

    def set_option(self, option: int, value: int) -> None:
        self._check(lib().micsa_set_option(self._ctx, option, value), "set_option")

    def kernel_name(self, algo: int) -> str:
        return lib().micsa_kernel_name(self._ctx, algo).decode()


def footprint(Lx: int, Ly: int, Lz: int, S: int = 1, R: int = 1, layout: int = LAYOUT_BYTE, gamma: int = 1) -> int:
    """Device bytes a pool job of this shape occupies."""
    out = ctypes.c_size_t()
    st = lib().micsa_pool_footprint(ctypes.byref(_params(Lx, Ly, Lz, S, R, layout, 0, gamma)), ctypes.byref(out))
    if st != OK:
        raise MicsaError(st, "micsa_pool_footprint")
    return out.value


class Pool:
    """Continuous-batching pool of annealing jobs (micsa_pool_*)."""

    def __init__(self, hbm_budget: int, max_running: int = 1 << 20, stream=None):
        self._pool = ctypes.c_void_p()
        st = lib().micsa_pool_create(int(hbm_budget), int(max_running), _stream_handle(stream),
                                     ctypes.byref(self._pool))
        if st != OK:
            raise MicsaError(st, "micsa_pool_create")
        self._jobs = {}

    def close(self) -> None:
        if self._pool:
            lib().micsa_pool_destroy(self._pool)
            self._pool = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str) -> None:
        if st != OK:
            raise MicsaError(st, f"{what}: {lib().micsa_status_string(st).decode()}")

    def submit(self, Lx, Ly, Lz, S, R, seed, sched: Schedule, layout: int = LAYOUT_BYTE, gamma: int = 1,
               lane_mode: int = LANES_SAMPLES) -> int:
        p = _params(Lx, Ly, Lz, S, R, layout, seed, gamma, lane_mode)
        cs, keep = _schedule_struct(sched)
        job = ctypes.c_int64()
        self._check(lib().micsa_pool_submit(self._pool, ctypes.byref(p), ctypes.byref(cs), ctypes.byref(job)),
                    "pool_submit")
        self._jobs[job.value] = (Lx, Ly, Lz, S, R, seed, gamma)
        return job.value

    def step(self, sweeps: int) -> tuple[int, int]:
        r, q = ctypes.c_int32(), ctypes.c_int32()
        self._check(lib().micsa_pool_step(self._pool, int(sweeps), ctypes.byref(r), ctypes.byref(q)), "pool_step")
        return r.value, q.value

    def sync(self) -> None:
        self._check(lib().micsa_pool_sync(self._pool), "pool_sync")

    def state(self, job: int) -> tuple[int, int]:
        st, k = ctypes.c_int32(), ctypes.c_int64()
        self._check(lib().micsa_pool_job_state(self._pool, job, ctypes.byref(st), ctypes.byref(k)), "job_state")
        return st.value, k.value

    def lattice(self, job: int) -> Lattice:
        ctx = ctypes.c_void_p()
        self._check(lib().micsa_pool_job_context(self._pool, job, ctypes.byref(ctx)), "job_context")
        return Lattice._borrow(ctx, *self._jobs[job])

    def release(self, job: int) -> None:
        self._check(lib().micsa_pool_release(self._pool, job), "pool_release")


class PT:
    """Parallel tempering of one Gaussian sample (micsa_pt_*, App. C): runs x 2
    replicas x M temperatures; arrays are by temperature, energies in units
    of the 2^-17 mesh."""

    def __init__(self, Lx: int, Ly: int, Lz: int, runs: int, T, J, seed: int, sweeps: int = 10,
                 algo: int = PT_WALKERS, houdayer: bool = True, stream=None):
        self.Lx, self.Ly, self.Lz, self.runs = Lx, Ly, Lz, runs
        self.N = Lx * Ly * Lz
        self.T = np.ascontiguousarray(T, np.float64)
        self.M = len(self.T)
        J = np.ascontiguousarray(J, np.float64)
        if J.size != 3 * self.N:
            raise ValueError(f"J must hold 3 x {self.N} couplings")
        self._ctx = ctypes.c_void_p()
        p = _PtParams(Lx, Ly, Lz, runs, self.M, sweeps, algo, int(bool(houdayer)), seed)
        st = lib().micsa_pt_create(ctypes.byref(p), _ptr(J), _ptr(self.T), _stream_handle(stream),
                                   ctypes.byref(self._ctx))
        if st != OK:
            raise MicsaError(st, f"micsa_pt_create({Lx},{Ly},{Lz}, runs={runs}, M={self.M}): "
                                 f"{lib().micsa_status_string(st).decode()}")

    def close(self) -> None:
        if self._ctx:
            lib().micsa_pt_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str) -> None:
        if st != OK:
            raise MicsaError(st, f"{what}: {lib().micsa_pt_last_error(self._ctx).decode()}")

    def step(self, n_emcs: int) -> None:
        self._check(lib().micsa_pt_step(self._ctx, int(n_emcs)), "pt_step")

    def sync(self) -> None:
        self._check(lib().micsa_pt_sync(self._ctx), "pt_sync")

    @property
    def emcs(self) -> int:
        e = ctypes.c_int64()
        self._check(lib().micsa_pt_get_emcs(self._ctx, ctypes.byref(e)), "pt_get_emcs")
        return e.value

    def read(self) -> tuple[np.ndarray, np.ndarray]:
        """(E [runs, 2, M], Q [runs, M]) by temperature."""
        E = np.zeros((self.runs, 2, self.M), np.int64)
        Q = np.zeros((self.runs, self.M), np.int64)
        self._check(lib().micsa_pt_read(self._ctx, _ptr(E), _ptr(Q)), "pt_read")
        return E, Q

    def spins(self) -> np.ndarray:
        s = np.zeros((self.runs, 2, self.M, self.N), np.uint8)
        self._check(lib().micsa_pt_read_spins(self._ctx, _ptr(s)), "pt_read_spins")
        return s

    def write_spins(self, sigma: np.ndarray) -> None:
        s = np.ascontiguousarray(sigma, np.uint8).reshape(self.runs, 2, self.M, self.N)
        self._check(lib().micsa_pt_write_spins(self._ctx, _ptr(s)), "pt_write_spins")

    def swaps(self) -> np.ndarray:
        w = np.zeros((self.runs, 2, self.M - 1), np.int64)
        self._check(lib().micsa_pt_read_swaps(self._ctx, _ptr(w)), "pt_read_swaps")
        return w

    def tables(self, kind: int, index: int) -> np.ndarray:
        t = np.zeros((4, 255), np.uint64)
        self._check(lib().micsa_pt_get_tables(self._ctx, int(kind), int(index), _ptr(t)), "pt_get_tables")
        return t

    def couplings(self) -> np.ndarray:
        Jq = np.zeros((3, self.N), np.int32)
        self._check(lib().micsa_pt_get_couplings(self._ctx, _ptr(Jq)), "pt_get_couplings")
        return Jq

    def set_kernel(self, kernel: int) -> None:
        self._check(lib().micsa_pt_set_kernel(self._ctx, int(kernel)), "pt_set_kernel")

    @property
    def kernel_name(self) -> str:
        return lib().micsa_pt_kernel_name(self._ctx).decode()

    def set_timing(self, on: bool) -> None:
        self._check(lib().micsa_pt_set_timing(self._ctx, int(bool(on))), "pt_set_timing")

    def timing(self, kind: int) -> tuple[float, int]:
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(lib().micsa_pt_get_timing(self._ctx, int(kind), ctypes.byref(ms), ctypes.byref(n)),
                    "pt_get_timing")
        return ms.value, n.value
