"""Launch-shape autotuner for the MicSA sweeps.

For a lattice shape it times candidate launch shapes with the library's
per-launch event timing (the best of two trials), rejects any candidate whose state after the trial
sweeps differs in a single bit from the per-half reference kernel (the
bit-exact gate: launch shapes must never change results), and returns the
fastest.  Three families:
  tune()            the fused byte sweep: tile rows TY x planes TZ, prefetch
                    depth, one or two sweeps per pass;
  tune_multispin()  the one-launch multispin sweep: tile rows and planes,
                    XCD tile order, one or two sweeps per pass;
  tune_bitplane()   the one-launch bit-plane sweep: planes per work-group,
                    refresh levels drawn ahead or in place.
Results are cached in a JSON file keyed by device, family and shape.

Only argument marshalling and timing happen here; all sweeps run in
libmicsa through the binding.
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import dataclass

import numpy as np

from . import micsa as M

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


@dataclass
class TileResult:
    ty: int
    tz: int
    us_per_sweep: float
    prefetch: int = 1
    temporal: int = 1


def _divisors(n: int, cap: int) -> list[int]:
    return [d for d in range(1, min(n, cap) + 1) if n % d == 0]


def candidates(Lx: int, Ly: int, Lz: int) -> list[tuple[int, int]]:
    nc = Lx // 32
    tys = [d for d in _divisors(Ly, 64) if (d + 4) * nc <= 1024 and d >= min(4, Ly)]
    tzs = [d for d in _divisors(Lz, 64) if d >= min(4, Lz)]
    # keep the grid reasonably small: powers of two and the largest admissible values
    def trim(v):
        keep = sorted({x for x in v if x & (x - 1) == 0} | set(v[-2:]))
        return keep
    return [(ty, tz) for ty in trim(tys) for tz in trim(tzs)]


def _device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:
        return "unknown"


def _state_digest(g: M.Lattice) -> str:
    """Spins, daemons and energy; the incremental tally where the path keeps
    one (the bit-plane per-half reference keeps none), else the from-scratch
    energy in its place."""
    h = hashlib.sha256()
    try:
        tally = g.energy_tally()
    except M.MicsaError:
        tally = g.energy()
    for a in (g.spins(), g.daemons(), g.energy(), tally):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _run(shape, seed, kernel, ty, tz, sweeps, warm, timed, prefetch=1, temporal=1, layout=M.LAYOUT_BYTE, opts=(),
         lane_mode=M.LANES_SAMPLES):
    Lx, Ly, Lz, S, R = shape
    g = M.Lattice(Lx, Ly, Lz, S, R, seed, layout=layout, lane_mode=lane_mode)
    try:
        g.set_option(M.OPT_SWEEP_KERNEL, kernel)
        if layout == M.LAYOUT_BYTE:
            g.set_option(M.OPT_PREFETCH, prefetch)
            g.set_option(M.OPT_TEMPORAL, temporal)
        for opt, v in opts:
            g.set_option(opt, v)
        if ty:
            g.set_option(M.OPT_TILE_Y, ty)
        if tz:
            g.set_option(M.OPT_TILE_Z, tz)
        g.set_schedule(M.Schedule(M.SCHED_CONST, 0.9, 0.9, warm + sweeps, 7))
        g.sweep(M.ALGO_MICSA, warm)
        g.sync()
        g.set_timing(timed)
        g.sweep(M.ALGO_MICSA, sweeps)
        ms, n = g.timing(M.TIME_SWEEP)
        return _state_digest(g), (ms / sweeps * 1e3 if n else float("nan"))
    finally:
        g.close()


def _timed(*args, trials: int = 2, **kw):
    """_run repeated: the state digest (every trial must agree) and the best
    time of the trials (one trial's time is noisy on short runs)."""
    out = [_run(*args, **kw) for _ in range(trials)]
    if len({d for d, _ in out}) != 1:
        raise RuntimeError("repeated trials of one launch shape gave different states")
    return out[0][0], min(us for _, us in out)


def tune(Lx: int, Ly: int, Lz: int, S: int = 1, R: int = 1, sweeps: int = 12, use_cache: bool = True,
         verbose: bool = False) -> TileResult:
    """Fastest bit-exact tile of the fused sweep for this lattice shape."""
    shape = (Lx, Ly, Lz, S, R)
    key = f"{_device_name()}|{Lx}x{Ly}x{Lz}|S{S}|R{R}"
    cache = {}
    if use_cache and os.path.exists(CACHE_PATH):
        with open(CACHE_PATH) as f:
            cache = json.load(f)
        if key in cache:
            return TileResult(**cache[key])
    seed = 0x7E57
    warm = 3
    ref, _ = _run(shape, seed, M.KERNEL_SIMPLE, 0, 0, sweeps, warm, False)
    best = None
    for ty, tz in candidates(Lx, Ly, Lz):
        for pf, tp in ((1, 1), (2, 1), (1, 2)):  # prefetch applies to one-sweep passes only
            digest, us = _timed(shape, seed, M.KERNEL_FUSED, ty, tz, sweeps, warm, True, pf, tp)
            if digest != ref:
                raise RuntimeError(f"tile TY={ty} TZ={tz} prefetch {pf} sweeps/pass {tp} changed the result: "
                                   f"the fused sweep is wrong for {shape}")
            if verbose:
                print(f"  TY={ty:3d} TZ={tz:3d} PF={pf} T={tp}: {us:9.2f} us/sweep", flush=True)
            if best is None or us < best.us_per_sweep:
                best = TileResult(ty, tz, us, pf, tp)
    if use_cache:
        cache[key] = best.__dict__
        with open(CACHE_PATH, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return best


@dataclass
class MultispinResult:
    ty: int
    tz: int
    xcd: int
    temporal: int
    us_per_sweep: float


def _cached(key):
    if os.path.exists(CACHE_PATH):
        with open(CACHE_PATH) as f:
            return json.load(f).get(key)
    return None


def _store(key, value):
    cache = {}
    if os.path.exists(CACHE_PATH):
        with open(CACHE_PATH) as f:
            cache = json.load(f)
    cache[key] = value
    with open(CACHE_PATH, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def multispin_candidates(Lx: int, Ly: int, Lz: int) -> list[tuple[int, int, int, int]]:
    """(TY, TZ, XCD order, sweeps per pass): the automatic tile (0, 0) and
    tiles whose lanes fill whole waves, z depths 4 / 8 / 16 dividing Lz, the
    three tile orders, one or two sweeps per pass."""
    W = Lx // 128
    out = [(0, 0, x, t) for t in (2, 1) for x in (2, 1, 0)]
    for t in (2, 1):
        ring = 4 * t
        for lanes in (128, 192, 256):
            ty = lanes // W - ring
            if 1 <= ty <= Ly and lanes % W == 0:
                for tz in (4, 8, 16):
                    if Lz % tz == 0:
                        out.append((ty, tz, 2, t))
    return list(dict.fromkeys(out))


def tune_multispin(Lx: int, Ly: int, Lz: int, S: int = 1, R: int = 1, sweeps: int = 16, use_cache: bool = True,
                   verbose: bool = False) -> MultispinResult:
    """Fastest bit-exact launch shape of the one-launch multispin sweep."""
    shape = (Lx, Ly, Lz, S, R)
    key = f"{_device_name()}|multispin|{Lx}x{Ly}x{Lz}|S{S}|R{R}"
    if use_cache and (hit := _cached(key)):
        return MultispinResult(**hit)
    seed, warm = 0x7E57, 2
    ref, _ = _run(shape, seed, M.KERNEL_SIMPLE, 0, 0, sweeps, warm, False)
    best = None
    for ty, tz, xcd, temporal in multispin_candidates(Lx, Ly, Lz):
        digest, us = _timed(shape, seed, M.KERNEL_MULTISPIN, ty, tz, sweeps, warm, True,
                            opts=((M.OPT_XCD_MAP, xcd), (M.OPT_MSC_PASS, temporal)))
        if digest != ref:
            raise RuntimeError(f"multispin TY={ty} TZ={tz} xcd {xcd} sweeps/pass {temporal} changed the result "
                               f"for {shape}")
        if verbose:
            print(f"  TY={ty:3d} TZ={tz:3d} XCD={xcd} T={temporal}: {us:9.2f} us/sweep", flush=True)
        if best is None or us < best.us_per_sweep:
            best = MultispinResult(ty, tz, xcd, temporal, us)
    if use_cache:
        _store(key, best.__dict__)
    return best


@dataclass
class BitplaneResult:
    tz: int
    draw_ahead: int
    us_per_sweep: float


def tune_bitplane(Lx: int, Ly: int, Lz: int, S: int, R: int, lane_mode: int = 0, sweeps: int = 40,
                  use_cache: bool = True, verbose: bool = False) -> BitplaneResult:
    """Fastest bit-exact launch of the one-launch bit-plane sweep: one or two
    planes per work-group, refresh levels drawn ahead or in place."""
    shape = (Lx, Ly, Lz, S, R)
    key = f"{_device_name()}|bitplane|{Lx}x{Ly}x{Lz}|S{S}|R{R}|lanes{lane_mode}"
    if use_cache and (hit := _cached(key)):
        return BitplaneResult(**hit)
    seed, warm = 0x7E57, 2
    ref, _ = _run(shape, seed, M.KERNEL_SIMPLE, 0, 0, sweeps, warm, False, layout=M.LAYOUT_BITPLANE,
                  lane_mode=lane_mode)
    best = None
    for tz in (1, 2):
        if Lz % tz:
            continue
        for ahead in (1, 0):
            digest, us = _timed(shape, seed, M.KERNEL_AUTO, 0, tz, sweeps, warm, True, layout=M.LAYOUT_BITPLANE,
                                opts=((M.OPT_DRAW_AHEAD, ahead),), lane_mode=lane_mode)
            if digest != ref:
                raise RuntimeError(f"bit-plane TZ={tz} draw-ahead {ahead} changed the result for {shape}")
            if verbose:
                print(f"  TZ={tz} ahead={ahead}: {us:9.2f} us/sweep", flush=True)
            if best is None or us < best.us_per_sweep:
                best = BitplaneResult(tz, ahead, us)
    if use_cache:
        _store(key, best.__dict__)
    return best
