"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/micsa.h, and rejects invalid arguments before touching
the device."""
import ctypes
import os
import re

import numpy as np

import pytest

from paper_2506_16240_amd import micsa as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^[A-Za-z_][\w\s\*]*?\b(micsa_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(M.LIB_PATH)
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    # and the binding wraps exactly those
    assert sorted(M.exported_symbols()) == declared


def test_status_strings():
    lib = M.lib()
    assert lib.micsa_status_string(0) == b"ok"
    for st in (-1, -2, -3, -4, -5):
        assert lib.micsa_status_string(st) not in (b"ok", b"unknown status")


@pytest.mark.parametrize("dims", [(7, 8, 8), (12, 8, 8), (4, 8, 8), (8, 3, 8), (8, 8, 1), (0, 8, 8), (8, 8, -2)])
def test_create_rejects_bad_sides(dims):
    p = M._params(*dims, 1, 1, 0, 1)
    out = ctypes.c_void_p(123)
    assert M.lib().micsa_create(ctypes.byref(p), None, ctypes.byref(out)) == M.EINVAL
    assert not out.value


@pytest.mark.parametrize("S,R,layout", [(0, 1, 0), (1, 0, 0), (1 << 24, 1, 0), (1, 1, 7)])
def test_create_rejects_bad_counts_and_layout(S, R, layout):
    p = M._params(8, 8, 8, S, R, layout, 1)
    out = ctypes.c_void_p()
    assert M.lib().micsa_create(ctypes.byref(p), None, ctypes.byref(out)) == M.EINVAL
    assert not out.value


@pytest.mark.parametrize("gamma,layout", [(7, 0), (-1, 0), (2, 1), (6, 1)])
def test_create_rejects_bad_gamma(gamma, layout):
    """gamma daemons per site: 1..6, and more than one only in the byte layout."""
    p = M._params(8, 8, 8, 1, 1, layout, 1, gamma)
    out = ctypes.c_void_p()
    assert M.lib().micsa_create(ctypes.byref(p), None, ctypes.byref(out)) == M.EINVAL
    assert not out.value
    size = ctypes.c_size_t()
    assert M.lib().micsa_pool_footprint(ctypes.byref(M._params(8, 8, 8, 1, 2, 0, 1, 3)), ctypes.byref(size)) == M.OK
    one = ctypes.c_size_t()
    assert M.lib().micsa_pool_footprint(ctypes.byref(M._params(8, 8, 8, 1, 2, 0, 1, 1)), ctypes.byref(one)) == M.OK
    assert size.value - one.value == 2 * 2 * 512 * 2  # two more families: 2 buffers x 2 lattices x N bytes each


def test_null_arguments():
    lib = M.lib()
    assert lib.micsa_create(None, None, None) == M.EINVAL
    assert lib.micsa_destroy(None) == M.OK
    assert lib.micsa_sweep(None, 0, 1) == M.EINVAL
    assert lib.micsa_sync(None) == M.EINVAL
    assert lib.micsa_read_energy(None, None) == M.EINVAL
    assert lib.micsa_set_schedule(None, None) == M.EINVAL
    assert lib.micsa_last_error(None) == b"null context"
    n = ctypes.c_size_t(0)
    assert lib.micsa_save(None, None, ctypes.byref(n)) == M.EINVAL
    assert lib.micsa_load(None, None, 0) == M.EINVAL


@pytest.mark.parametrize("layout,lane_mode", [(0, 2), (1, -1), (0, 1)])
def test_create_rejects_bad_lane_mode(layout, lane_mode):
    """Lane modes exist for the bit-plane layout only."""
    p = M._params(8, 8, 8, 1, 2, layout, 1, 1, lane_mode)
    out = ctypes.c_void_p()
    assert M.lib().micsa_create(ctypes.byref(p), None, ctypes.byref(out)) == M.EINVAL
    assert not out.value


def test_params_struct_layout():
    """lane_mode sits in the padding before the 64-bit seed: the struct keeps
    its size and the seed its offset."""
    assert ctypes.sizeof(M._Params) == 40
    assert M._Params.seed.offset == 32 and M._Params.lane_mode.offset == 28


def _pt_create(Lx=4, Ly=4, Lz=4, runs=1, T=(0.5, 1.0), J=None, sweeps=10, algo=0, houdayer=1):
    N = Lx * Ly * Lz
    J = np.zeros(3 * N) if J is None else np.asarray(J, np.float64)
    T = np.asarray(T, np.float64)
    p = M._PtParams(Lx, Ly, Lz, runs, len(T), sweeps, algo, houdayer, 1)
    ctx = ctypes.c_void_p()
    st = M.lib().micsa_pt_create(ctypes.byref(p), J.ctypes.data, T.ctypes.data, None, ctypes.byref(ctx))
    return st, ctx


@pytest.mark.parametrize("kw", [dict(Lx=5), dict(Ly=3), dict(Lz=0), dict(Lx=66, Ly=2, Lz=2), dict(Lx=32, Ly=32, Lz=32),
                                dict(runs=0), dict(runs=1 << 24), dict(T=(1.0,)), dict(T=tuple(np.linspace(1, 2, 65))),
                                dict(sweeps=0), dict(sweeps=65), dict(algo=2), dict(houdayer=2),
                                dict(T=(1.0, 1.0)), dict(T=(1.0, 0.5)), dict(T=(-1.0, 1.0)), dict(T=(0.5, np.inf)),
                                dict(T=(0.5, 1000.0)), dict(T=(1.0, 1.00001))])
def test_pt_create_rejects_bad_arguments(kw):
    """Invalid shapes, counts, ladders (not increasing, walkers too hot for
    32 bits, exchange rates too small for four digits) are refused before
    any device work."""
    st, ctx = _pt_create(**kw)
    assert st == M.EINVAL and not ctx


@pytest.mark.parametrize("bad", [8.5, float("nan"), float("inf")])
def test_pt_create_rejects_bad_couplings(bad):
    J = np.zeros(3 * 64)
    J[17] = bad
    st, ctx = _pt_create(J=J)
    assert st == M.EINVAL and not ctx


def test_binding_constants_match_the_header():
    """Every MICSA_OPT_* / MICSA_KERNEL_* value the header declares has the
    same value in the Python binding (a mismatch would set the wrong option)."""
    text = open(os.path.join(ROOT, "include", "micsa.h")).read()
    pairs = re.findall(r"\bMICSA_((?:OPT|KERNEL|LANES|LAYOUT)_[A-Z0-9_]+)\s*=\s*(\d+)", text)
    assert len(pairs) >= 14
    for name, value in pairs:
        assert getattr(M, name) == int(value), name


def test_pool_footprint_counts_the_multispin_planes():
    """A byte-layout job whose rows split into 128-site words may run on the
    multispin planes, which its first long MicSA call allocates: spin, two
    level planes, their alternates, two drawn-level planes and the six
    coupling planes of the even sites, 11/8 B per site per lattice, on top of
    the byte state.  Same N and lattice count, one eligible and one not."""
    def fp(*shape, gamma=1):
        out = ctypes.c_size_t()
        assert M.lib().micsa_pool_footprint(ctypes.byref(M._params(*shape, 0, 1, gamma)), ctypes.byref(out)) == M.OK
        return out.value
    for S, R in ((1, 1), (2, 3)):
        N, L = 128 * 8 * 8, S * R
        assert fp(128, 8, 8, S, R) - fp(64, 16, 8, S, R) == 11 * L * N // 8
    # gamma > 1 never runs multispin
    assert fp(128, 8, 8, 1, 1, gamma=2) - fp(64, 16, 8, 1, 1, gamma=2) == 0


def test_pool_footprint_counts_the_slab_levels():
    """A byte-layout job on the slab sweep (too large for the resident
    sweep, Lx < 128) draws refresh levels ahead into two buffers of a byte
    per site per lattice; a resident-size lattice and a gamma > 1 one do
    not."""
    def fp(*shape, gamma=1):
        out = ctypes.c_size_t()
        assert M.lib().micsa_pool_footprint(ctypes.byref(M._params(*shape, 0, 1, gamma)), ctypes.byref(out)) == M.OK
        return out.value
    N, L = 64 ** 3, 2
    base = 2 * L * N * 2 + (L + 1) * 64 * 8  # two state buffers of spin + daemon bytes, and the slots
    assert fp(64, 64, 64, 1, 2) - base == 2 * L * N
    assert fp(32, 32, 32, 1, 2) == 2 * L * 32 ** 3 * 2 + (L + 1) * 64 * 8  # resident: no drawn levels
    assert fp(64, 64, 64, 1, 2, gamma=2) == 2 * L * N * 3 + (L + 1) * 64 * 8
