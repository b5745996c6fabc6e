#!/usr/bin/env python3
"""Spin updates/ns of MicSA and of the heat-bath and Metropolis baselines on one MI355X.

Workload (default): the large anneal -- one 512^3 lattice (134M spins) of the
3D EA +-J model (byte arrays at the library's boundary, swept on multispin
bit planes), linear schedule T = 3.0 -> 0.2 over 10^4 sweeps, daemon refresh
every 20 sweeps.  A step is one refresh period: the refresh and 20 sweeps
(even half + odd half each, with the incremental energy tally).  --steps 500
is the whole anneal.  The heat bath and Metropolis run
the same steps on lattices from the same seed.  Prints one JSON line.

--workload pt_gauss_L10_200x2x40: the equilibrium workload of App. C
(parallel tempering of a Gaussian sample, L = 10, 200 runs x 2 replicas x
40 temperatures, 10 sweeps per EMCS, Houdayer moves); a step is one EMCS;
walkers against the Metropolis update.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# Algorithmic bytes per site and pass over the state (one sweep, or two with
# the two-sweep fused kernel; byte layout):
# spin byte read+write 2 B (an even site's byte also holds its six bond bits,
# so the couplings ride along at no cost), daemon read+write 2 B.  The
# baselines move the spin bytes only (plus one 32-bit uniform per update,
# generated in registers).
BYTES_PER_UPDATE = {"micsa": 4.0, "heatbath": 2.0, "metropolis": 2.0, "walkers": 4.0}
# Walkers (Sec. 2.6) on the fused sweep: each timestep's wandering is applied
# by the next sweep as it loads the daemons (a byte shift across the two
# parity arrays of a row), so a walker sweep moves the same 4 B per site as a
# daemon sweep.  (On the per-half path a separate wandering kernel reads and
# writes every daemon byte once more.)
# Bit-plane layout (64 samples per 64-bit word): spin word read+write 16 B,
# two daemon planes read+write 32 B, three forward-bond planes 24 B shared by
# the two replicas of a sample: (16 + 32 + 12) / 64 = 0.9375 B per update.
BYTES_PER_UPDATE_BITPLANE = 0.9375
# Multispin planes of one lattice (64 sites of a row per word): spin bit read
# and written, two daemon bits read and written, and the three couplings per
# site (six per even site) read once per sweep: 9 bits = 1.125 B per update.
BYTES_PER_UPDATE_MULTISPIN = 1.125


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2506_16240_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(name)
    if not e or e.get("kernel_hash") != kernel_hash():
        return None
    return e.get("bytes_per_launch")


def tile_options(tile):
    """Launch options of a tile: a dict {option: value} (from the tuner) or a
    tuple (TY, TZ[, PREFETCH[, SWEEPS_PER_PASS]])."""
    from paper_2506_16240_amd import micsa as M

    if not tile:
        return []
    if isinstance(tile, dict):
        return [(getattr(M, k), v) for k, v in tile.items()]
    names = (M.OPT_TILE_Y, M.OPT_TILE_Z, M.OPT_PREFETCH, M.OPT_TEMPORAL)
    return list(zip(names, tile))


def run_gpu(w, algo_name: str, steps: int, warmup: int, stream, tile=None, layout: int = 0, events: bool = False,
            gamma: int = 1, period=None, c4: int = 0, kernel: int = 0):
    """One timed region of `steps` steps on a fresh lattice.  With events the
    library brackets every launch with a HIP event pair (per-kernel
    durations for the roofline); without, the region is timed as a whole
    (the throughput), since per-launch events slow launch-bound paths."""
    from paper_2506_16240_amd import micsa as M
    import torch

    def configure(lat):
        if kernel:
            lat.set_option(M.OPT_SWEEP_KERNEL, kernel)
        if algo_name == "micsa":
            for opt, v in tile_options(tile):
                lat.set_option(opt, v)

    algo = {"micsa": M.ALGO_MICSA, "heatbath": M.ALGO_HEATBATH, "metropolis": M.ALGO_METROPOLIS,
            "walkers": M.ALGO_WALKERS}[algo_name]
    sched = M.Schedule(w.kind, w.T0, w.T1, w.n_sweeps, w.period if period is None else period)
    P = w.period
    if warmup > 0:
        with M.Lattice(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed, stream=stream.cuda_stream, layout=layout,
                       gamma=gamma) as lw:
            configure(lw)
            lw.set_schedule(sched)
            lw.sweep(algo, warmup * P)
            lw.sync()
    lat = M.Lattice(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed, stream=stream.cuda_stream, layout=layout, gamma=gamma)
    configure(lat)
    lat.set_schedule(sched)
    lat.set_timing(events)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    lat.sweep(algo, steps * P)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    kind = {M.ALGO_MICSA: M.TIME_SWEEP, M.ALGO_HEATBATH: M.TIME_HEATBATH, M.ALGO_METROPOLIS: M.TIME_METROPOLIS,
            M.ALGO_WALKERS: M.TIME_SWEEP}[algo]
    k_ms, k_n = lat.timing(kind)
    r_ms, r_n = lat.timing(M.TIME_REFRESH)
    # property that holds at any size: the incremental tally (per lattice; per
    # lane of the bit-plane words) equals the from-scratch energy
    E = lat.energy()
    ok = bool((E == lat.energy_tally()).all())
    name = lat.kernel_name(algo)
    c4_ms = None
    if c4 > 0 and w.R >= 2:  # C4(r) sums of the final state (Sec. 3), timed as a whole
        lat.c4_sums()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(c4):
            lat.c4_sums()
        c4_ms = (time.perf_counter() - t) * 1e3 / c4
    lat.close()
    return {"ms": ms, "kernel_ms": k_ms, "kernel_launches": k_n, "refresh_ms": r_ms, "refresh_launches": r_n,
            "tally_check": ok, "kernel": name, "E_final": int(E[0]), "c4_ms": c4_ms}


def cpu_baseline(w, seconds: float, configure_gpu=None, stream=None, single_core_seconds: float = 8.0):
    """The CPU oracle on a bounded sample of the same workload (sweep loop
    only, all host threads, then one thread), and a parity check: the GPU
    path runs the same first K sweeps in one call with the launch options of
    the timed region, and its spins, daemons, energy and daemon energy must
    equal the oracle's bit for bit."""
    from oracle import oracle as O

    lat = O.Lattice(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
    sched = O.Schedule(w.kind, w.T0, w.T1, w.n_sweeps, w.period)
    sweeps = 0
    t = time.perf_counter()
    while True:
        lat.run(O.ALGO_MICSA, sched, 1, 0)
        sweeps += 1
        el = time.perf_counter() - t
        if el >= seconds or sweeps >= w.n_sweeps:
            break
    upd = w.N * w.lattices * sweeps
    out = {"value": round(upd / (el * 1e9), 4), "unit": "spin updates/ns", "cores": O.threads(),
           "kind": "oracle",
           "sample": f"MicSA sweeps 0..{sweeps - 1} of {w.name} ({sweeps} x {w.N * w.lattices} updates, "
                     f"{el:.1f} s, init excluded)"}
    parity = None
    if configure_gpu is not None:
        from paper_2506_16240_amd import micsa as M
        g = M.Lattice(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed, stream=stream.cuda_stream)
        configure_gpu(g)
        g.set_schedule(M.Schedule(w.kind, w.T0, w.T1, w.n_sweeps, w.period))
        g.sweep(M.ALGO_MICSA, sweeps)
        same = (np.array_equal(g.spins(), lat.sigma) and np.array_equal(g.daemons(), lat.m)
                and np.array_equal(g.energy(), lat.energy()) and np.array_equal(g.daemon_energy(), lat.daemon_energy())
                and np.array_equal(g.energy_tally(), lat.energy()))
        parity = {"sweeps": sweeps, "calls": 1, "kernel": g.kernel_name(M.ALGO_MICSA), "bit_exact": bool(same)}
        g.close()
    del lat
    # one core: the same sweeps from the start on one thread
    n_all = O.threads()
    O.set_threads(1)
    try:
        lat1 = O.Lattice(w.Lx, w.Ly, w.Lz, w.S, w.R, w.seed)
        s1 = 0
        t = time.perf_counter()
        while True:
            lat1.run(O.ALGO_MICSA, sched, 1, 0)
            s1 += 1
            el1 = time.perf_counter() - t
            if el1 >= single_core_seconds or s1 >= w.n_sweeps:
                break
        del lat1
    finally:
        O.set_threads(n_all)
    out["single_core"] = {"value": round(w.N * w.lattices * s1 / (el1 * 1e9), 4), "unit": "spin updates/ns",
                          "cores": 1, "sample": f"MicSA sweeps 0..{s1 - 1} of {w.name} ({el1:.1f} s)"}
    return out, parity


def copy_rate_gbs(stream, gib: float = 2.0, reps: int = 5) -> float:
    """Device-to-device copy rate (bytes read + bytes written per second, GB/s),
    the best of a few copies of `gib` GiB: the practical HBM ceiling beside
    the 8 TB/s vendor figure."""
    import torch

    n = int(gib * (1 << 30))
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        b.copy_(a)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        best = ms if best is None else min(best, ms)
    del a, b
    return 2.0 * n / (best * 1e6)


# Parallel tempering (App. C): the EMCS kernel is bound by integer VALU work
# in LDS, not by HBM (the spin rows of a clone are 800 B).  Algorithmic
# operations per spin update of the uncapped Creutz move: six sign
# applications and five additions for the local field, dH = 2 s h, n - dH,
# the acceptance compare and the two selects (walker, spin): 16 int32 ops.
# Peak: 256 CUs x 64 int32 lanes per clock x 2.4 GHz = 39.3 Tops/s.
PT_OPS_PER_UPDATE = 16
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def run_pt(w, algo: int, steps: int, warmup: int, stream, events: bool = False):
    from paper_2506_16240_amd import micsa as M
    import torch

    T, J = w.temperatures(), w.couplings()
    if warmup > 0:
        g = M.PT(w.L, w.L, w.L, w.runs, T, J, w.seed, w.sweeps, algo, True, stream=stream.cuda_stream)
        g.step(warmup)
        g.sync()
        g.close()
    g = M.PT(w.L, w.L, w.L, w.runs, T, J, w.seed, w.sweeps, algo, True, stream=stream.cuda_stream)
    g.set_timing(events)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    g.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    k_ms, k_n = g.timing(M.PT_TIME_EMCS)
    s_ms, s_n = g.timing(M.PT_TIME_SWAP)
    E, Q = g.read()
    sw = g.swaps()
    name = g.kernel_name
    g.close()
    N = w.N
    return {"ms": ms, "kernel_ms": k_ms, "kernel_launches": k_n, "swap_ms": s_ms, "swap_launches": s_n,
            "e_lowT": float(E[:, :, 0].mean()) * 2.0 ** -17 / N, "absq_lowT": float(abs(Q[:, 0]).mean()) / N,
            "swap_rate": float(sw.sum()) / (sw.size * steps), "kernel": name}


def pt_cpu_baseline(w, seconds: float):
    """The oracle on a bounded sample of the tempering workload: EMCS of the
    first few runs (the runs are independent)."""
    from oracle import oracle as O

    runs = 8
    lat = O.PTLattice(w.L, w.L, w.L, runs=runs, T=w.temperatures(), J=w.couplings(), seed=w.seed, sweeps=w.sweeps)
    n = 0
    t = time.perf_counter()
    while True:
        lat.run(1)
        n += 1
        el = time.perf_counter() - t
        if el >= seconds:
            break
    upd = w.N * 2 * w.M * runs * w.sweeps * n
    return {"value": round(upd / (el * 1e9), 4), "unit": "spin updates/ns", "cores": O.threads(), "kind": "oracle",
            "sample": f"{n} EMCS of runs 0..{runs - 1} of {w.name} ({upd} updates, {el:.1f} s, walkers)"}


def bench_pt(w, args) -> int:
    from paper_2506_16240_amd import micsa as M
    import torch

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    steps = args.steps
    updates = w.updates(steps)
    log(f"walkers: {w.name}, {steps} EMCS")
    wk = run_pt(w, M.PT_WALKERS, steps, args.warmup, stream)
    log(f"walkers: {wk['ms']:.1f} ms")
    wke = run_pt(w, M.PT_WALKERS, steps, 0, stream, events=True)
    mp = None
    if not args.no_metropolis:
        log(f"metropolis: {w.name}, {steps} EMCS")
        mp = run_pt(w, M.PT_METROPOLIS, steps, args.warmup, stream)
        log(f"metropolis: {mp['ms']:.1f} ms")
    avg_ms = wke["kernel_ms"] / wke["kernel_launches"]
    ops_launch = PT_OPS_PER_UPDATE * w.updates(1)
    achieved = ops_launch / (avg_ms * 1e9)  # Tops/s
    out = {
        "metric": "spin updates/ns (walkers vs Metropolis, parallel tempering, 1 GPU) + % of int32 VALU peak",
        "value": round(updates / (wk["ms"] * 1e6), 2),
        "unit": "spin updates/ns",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(wk["ms"] / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": w.name, "L": [w.L] * 3, "runs": w.runs, "replicas": 2, "temperatures": w.M,
                   "T": [w.Tmin, w.Tmax], "sweeps_per_emcs": w.sweeps, "houdayer": True, "step": "one EMCS"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 1),
                     "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                     "kernel": wke["kernel"], "avg_launch_ms": round(avg_ms, 5), "ops_per_launch": ops_launch,
                     "ops_per_update": PT_OPS_PER_UPDATE, "launches": wke["kernel_launches"],
                     "swap_kernel_avg_ms": round(wke["swap_ms"] / max(wke["swap_launches"], 1), 5)},
        "observables": {"e_at_Tmin": round(wk["e_lowT"], 5), "absq_at_Tmin": round(wk["absq_lowT"], 4),
                        "exchange_rate": round(wk["swap_rate"], 4)},
    }
    if mp is not None:
        out["metropolis"] = {"value": round(updates / (mp["ms"] * 1e6), 2), "unit": "spin updates/ns",
                             "ms_per_step": round(mp["ms"] / steps, 4)}
        out["walkers_over_metropolis"] = round(mp["ms"] / wk["ms"], 3)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = pt_cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="anneal_L512_T3.0-0.2")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the GPU run of the oracle's sample that is compared with it bit for bit")
    ap.add_argument("--no-heatbath", action="store_true")
    ap.add_argument("--no-metropolis", action="store_true")
    ap.add_argument("--no-walkers", action="store_true",
                    help="skip the walker leg (MicSA with forward-X wandering walkers, the paper's Table 3 variant)")
    ap.add_argument("--layout", choices=("byte", "bitplane"), default="byte",
                    help="MicSA layout (the baselines always run in the byte layout)")
    ap.add_argument("--tile", default="tune",
                    help="launch shape: 'tune' (autotuner, bit-exact gated), 'auto' (library default), "
                         "TY,TZ[,PREFETCH[,SWEEPS_PER_PASS]] (fused sweep) or library options by name, "
                         "e.g. OPT_TILE_Y=24,OPT_TILE_Z=16,OPT_MSC_PASS=2")
    ap.add_argument("--algo", choices=("micsa", "walkers"), default="micsa",
                    help="daemons (default) or walkers wandering every timestep (Sec. 2.6)")
    ap.add_argument("--gamma", type=int, default=1, help="daemons (walkers) per site (Sec. 2.8)")
    ap.add_argument("--kernel", choices=("auto", "fused", "multispin", "slab", "simple"), default="auto",
                    help="MicSA sweep kernel: library choice, the fused byte sweep, multispin bit planes, the "
                         "one-launch slab sweep or the per-half kernels")
    ap.add_argument("--hb-kernel", choices=("auto", "fused", "simple"), default="auto",
                    help="kernel of the heat-bath and Metropolis legs (library choice by default)")
    ap.add_argument("--refresh", choices=("period", "log2"), default="period",
                    help="refresh every period of the workload, or before every sweep t with t + 1 a power "
                         "of two (the procedure of Sec. 2.8.1: refresh, 2^s steps, refresh, ...)")
    ap.add_argument("--c4", type=int, default=0,
                    help="after the MicSA run, time this many C4(r) evaluations of the final state (R >= 2)")
    ap.add_argument("--copy-ref-gib", type=float, default=0.0,
                    help="after the run, copy this many GiB device-to-device (reference for HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: every lattice here fits one MI355X and the multi-GPU "
              "decomposition is not built (run with --gpus 1)", file=sys.stderr)
        return 2

    from paper_2506_16240_amd import micsa as M
    from paper_2506_16240_amd import workloads as W
    import torch

    if args.workload == W.PT_L10.name:
        return bench_pt(W.PT_L10, args)
    if args.workload not in W.ALL:
        print(f"unknown workload {args.workload}; one of {sorted(W.ALL) + [W.PT_L10.name]}", file=sys.stderr)
        return 2
    w = W.ALL[args.workload]
    steps = args.steps
    if steps * w.period > w.n_sweeps:
        print(f"--steps {steps} exceeds the {w.n_sweeps}-sweep schedule", file=sys.stderr)
        return 2
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    sweeps = steps * w.period
    updates = w.N * w.lattices * sweeps

    layout = 1 if args.layout == "bitplane" else 0
    fused = layout == 0 and w.Lx % 32 == 0 and w.Lx >= 128
    # MicSA on the multispin planes (the library's choice for long calls on
    # lattices with Lx % 128 == 0): the tuner picks its tile, tile order and
    # sweeps per pass
    multispin = (layout == 0 and args.kernel in ("auto", "multispin") and w.Lx % 128 == 0 and args.gamma == 1
                 and args.algo == "micsa" and w.N * 3 > 150 * 1024 * 2)
    tile = None
    if args.tile == "tune" and args.algo == "micsa" and args.gamma == 1:
        # warm-up: the tuner times launch shapes of the path this workload runs
        # (bit-exact gate against the per-half kernels); cached per device and shape
        from paper_2506_16240_amd import tune
        if multispin:
            log("tuning the multispin sweep (tile, XCD order, sweeps per pass)")
            best = tune.tune_multispin(w.Lx, w.Ly, w.Lz, w.S, w.R)
            tile = {"OPT_TILE_Y": best.ty, "OPT_TILE_Z": best.tz, "OPT_XCD_MAP": best.xcd,
                    "OPT_MSC_PASS": best.temporal}
            log(f"multispin TY={best.ty} TZ={best.tz} xcd {best.xcd} sweeps/pass {best.temporal} "
                f"({best.us_per_sweep:.2f} us/sweep in tuning)")
        elif layout:
            log("tuning the bit-plane sweep (planes per work-group, draw ahead)")
            best = tune.tune_bitplane(w.Lx, w.Ly, w.Lz, w.S, w.R)
            tile = {"OPT_TILE_Z": best.tz, "OPT_DRAW_AHEAD": best.draw_ahead}
            log(f"bit-plane TZ={best.tz} draw-ahead {best.draw_ahead} ({best.us_per_sweep:.2f} us/sweep in tuning)")
        elif fused:
            log("tuning fused-sweep tiles")
            best = tune.tune(w.Lx, w.Ly, w.Lz, w.S, w.R, use_cache=False)
            tile = (best.ty, best.tz, best.prefetch, best.temporal)
            log(f"tile TY={best.ty} TZ={best.tz} prefetch {best.prefetch} sweeps/pass {best.temporal} "
                f"({best.us_per_sweep:.1f} us/sweep in tuning)")
    elif args.tile not in ("auto", "tune") and "=" in args.tile:
        # library options by name, e.g. OPT_TILE_Y=24,OPT_TILE_Z=16,OPT_MSC_PASS=2
        tile = {k.strip(): int(v) for k, v in (kv.split("=") for kv in args.tile.split(","))}
        for k in tile:
            if not (k.startswith("OPT_") and hasattr(M, k)):
                print(f"--tile: unknown option {k}", file=sys.stderr)
                return 2
    elif args.tile not in ("auto", "tune"):
        tile = tuple(int(v) for v in args.tile.split(","))
    algo_name = args.algo
    period = M.REFRESH_LOG2 if args.refresh == "log2" else None
    if args.gamma != 1 and (layout or tile):
        tile = None  # gamma > 1 runs the per-half kernels
    log(f"{algo_name}: {w.name}, {sweeps} sweeps, gamma {args.gamma}, refresh {args.refresh}")
    kern = {"auto": 0, "fused": M.KERNEL_FUSED, "multispin": M.KERNEL_MULTISPIN, "slab": M.KERNEL_SLAB,
            "simple": M.KERNEL_SIMPLE}[args.kernel]
    hb_kern = {"auto": 0, "fused": M.KERNEL_FUSED, "simple": M.KERNEL_SIMPLE}[args.hb_kernel]
    mi = run_gpu(w, algo_name, steps, args.warmup, stream, tile, layout, gamma=args.gamma, period=period,
                 c4=args.c4, kernel=kern)
    log(f"{algo_name}: {mi['ms']:.1f} ms, tally check {mi['tally_check']}")
    log(f"{algo_name} again with per-launch events (kernel durations)")
    mk = run_gpu(w, algo_name, steps, 0, stream, tile, layout, events=True, gamma=args.gamma, period=period,
                 kernel=kern)
    log(f"micsa with events: {mk['ms']:.1f} ms, {mk['kernel_launches']} launches")
    hb = None
    if not args.no_heatbath:
        log(f"heatbath: {w.name}, {sweeps} sweeps")
        hb = run_gpu(w, "heatbath", steps, args.warmup, stream, kernel=hb_kern)
        log(f"heatbath: {hb['ms']:.1f} ms")
    mp = None
    if not args.no_metropolis:
        log(f"metropolis: {w.name}, {sweeps} sweeps")
        mp = run_gpu(w, "metropolis", steps, args.warmup, stream, kernel=hb_kern)
        log(f"metropolis: {mp['ms']:.1f} ms")
    wk = None
    if not args.no_walkers and algo_name == "micsa" and args.gamma == 1 and not layout:
        log(f"walkers: {w.name}, {sweeps} sweeps")
        wk = run_gpu(w, "walkers", steps, args.warmup, stream, tile, layout, period=period)
        log(f"walkers: {wk['ms']:.1f} ms")

    value = updates / (mi["ms"] * 1e6)
    # dominant kernel: the sweep kernel.  A launch covers one half sweep
    # (per-half kernels), one sweep, or two sweeps in one pass over the state;
    # the algorithmic bytes per launch are those of one pass over the sites
    # it touches: bytes per update x sites x min(1, sweeps per launch).
    # The average launch duration is the timed region (HIP events on the
    # library's stream around the whole region, no per-launch events) over its
    # launches: an upper bound on the kernel's own duration, since the region
    # also holds the gaps between launches and any other kernel of the path.
    # Per-launch events (the second region) slow the launches and include
    # dispatch latency; their average is reported beside it.
    sweeps_per_launch = sweeps / mk["kernel_launches"]
    avg_ms = mi["ms"] / mk["kernel_launches"]
    event_ms = mk["kernel_ms"] / mk["kernel_launches"]
    per_update = BYTES_PER_UPDATE_BITPLANE if layout else BYTES_PER_UPDATE[algo_name]
    if "k_wander" in mi["kernel"]:  # a separate wandering kernel moves every daemon byte once more
        per_update += 2.0
    if mi["kernel"] in ("k_msc_half", "k_msc_sweep", "k_msc_sweep_multi"):
        per_update = BYTES_PER_UPDATE_MULTISPIN
    bytes_launch = per_update * w.N * w.lattices * min(1.0, sweeps_per_launch)
    achieved = bytes_launch / (avg_ms * 1e6)  # GB/s
    traffic = measured_traffic(mi["kernel"])
    # what the timed kernel computes on: the multispin sweep holds 1-bit
    # spin and coupling planes and 2-bit daemons as two planes (64 sites per
    # 64-bit word); the bit-plane layout the same with 64 samples per word;
    # the byte kernels one byte per spin and per daemon
    if mi["kernel"].startswith("k_msc"):
        layout_name, dtype = "multispin", "u1 bit planes (2-bit daemons)"
    elif layout:
        layout_name, dtype = "bitplane", "u1 bit planes (2-bit daemons)"
    else:
        layout_name, dtype = "byte", "u8"
    out = {
        "metric": "spin updates/ns (MicSA vs heat-bath, 1 GPU) + % of HBM roofline",
        "algo": algo_name,
        "value": round(value, 2),
        "unit": "spin updates/ns",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(mi["ms"] / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "L": [w.Lx, w.Ly, w.Lz], "samples": w.S, "replicas": w.R,
                   "sweeps_per_step": w.period, "sweeps": sweeps, "schedule": f"T {w.T0}->{w.T1}",
                   "layout": layout_name, "kernel": mi["kernel"],
                   "tile": (tile if isinstance(tile, dict) else list(tile)) if tile else "auto",
                   "gamma": args.gamma, "refresh": args.refresh},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": mi["kernel"], "avg_launch_ms": round(avg_ms, 5),
                     "event_launch_ms": round(event_ms, 5),
                     "bytes_per_launch": bytes_launch, "launches": mk["kernel_launches"],
                     "sweeps_per_launch": round(sweeps_per_launch, 3),
                     "bytes_per_update": round(bytes_launch / (sweeps_per_launch * w.N * w.lattices), 3),
                     # the HBM rate a kernel making one sweep per pass over the
                     # state (per_update bytes per update) would need for the
                     # same throughput; above 1 when two sweeps per pass beat the
                     # one-sweep ceiling
                     "one_sweep_equivalent": {"bytes_per_update": per_update,
                                              "GBs": round(value * per_update, 1),
                                              "frac": round(value * per_update / HBM_PEAK_GBS, 4)}},
        "checks": {"micsa_tally_equals_energy": mi["tally_check"]},
    }
    if mi["c4_ms"] is not None:
        nbytes = w.N * w.lattices  # spin bytes read per evaluation
        out["c4"] = {"ms_per_evaluation": round(mi["c4_ms"], 4), "spin_bytes": nbytes,
                     "GB_per_s": round(nbytes / (mi["c4_ms"] * 1e6), 1)}
    if hb is not None:
        out["heatbath"] = {"value": round(updates / (hb["ms"] * 1e6), 2), "unit": "spin updates/ns",
                           "ms_per_step": round(hb["ms"] / steps, 4), "kernel": hb["kernel"]}
        out["micsa_over_heatbath"] = round(hb["ms"] / mi["ms"], 3)
        out["checks"]["heatbath_tally_equals_energy"] = hb["tally_check"]
    if mp is not None:
        out["metropolis"] = {"value": round(updates / (mp["ms"] * 1e6), 2), "unit": "spin updates/ns",
                             "ms_per_step": round(mp["ms"] / steps, 4), "kernel": mp["kernel"]}
        out["micsa_over_metropolis"] = round(mp["ms"] / mi["ms"], 3)
        out["checks"]["metropolis_tally_equals_energy"] = mp["tally_check"]
    if wk is not None:
        out["walkers"] = {"value": round(updates / (wk["ms"] * 1e6), 2), "unit": "spin updates/ns",
                          "ms_per_step": round(wk["ms"] / steps, 4), "kernel": wk["kernel"]}
        out["checks"]["walkers_tally_equals_energy"] = wk["tally_check"]
        if mp is not None:
            out["walkers_over_metropolis"] = round(mp["ms"] / wk["ms"], 3)
    copy_gbs = copy_rate_gbs(stream)
    out["roofline"]["copy_GBs"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / copy_gbs, 4)
    if args.copy_ref_gib > 0:
        n = int(args.copy_ref_gib * (1 << 30))
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cfg = None
        if not args.no_parity and algo_name == "micsa" and args.gamma == 1 and not layout:
            def cfg(lat):
                lat.set_option(M.OPT_SWEEP_KERNEL, kern)
                for opt, v in tile_options(tile):
                    lat.set_option(opt, v)
        cb, parity = cpu_baseline(w, args.cpu_seconds, cfg, stream)
        out["cpu_baseline"] = cb
        if parity is not None:
            out["checks"]["oracle_parity_K"] = parity
            log(f"oracle parity over the first {parity['sweeps']} sweeps: {parity['bit_exact']}")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
