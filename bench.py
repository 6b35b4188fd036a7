#!/usr/bin/env python3
"""Benchmark of the fused fluctuating central-moment LBM step on one MI355X.

Workload (the headline one): D3Q27, 256^3 periodic box, rho0 = 1, tau = 0.8,
kT = 1e-4, Philox seed 1, started at rest; populations stored as FP32
deviations f_i - w_i rho0, FP32 collision, per-step FP64 statistics.  A step
is one pass of the whole path: pull streaming, moments, noise, collision,
back transformation, store, and the statistics reduction.

Prints one JSON line with the throughput in GLUPS (10^9 lattice-site updates
per second), the HBM roofline of the fused-step kernel, FP16/BF16-storage
variants and their <u^2> deviation from the FP32 run (same noise), and the
CPU oracle's throughput on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

Q = 27
SHAPE = (256, 256, 256)
TAU, KT, RHO0, SEED = 0.8, 1e-4, 1.0, 1
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published


def bytes_per_site(storage, q=Q):
    # every population read once and written once per step
    return 2 * q * {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[storage]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_2602_16486_amd/csrc/cmflb_step.h",
                  "paper_2602_16486_amd/csrc/cmflb_step_pull.hip",
                  "paper_2602_16486_amd/csrc/cmflb_device.h",
                  "paper_2602_16486_amd/csrc/cmflb_internal.h",
                  "paper_2602_16486_amd/csrc/cmflb_d3q19.h")
COUNTERS = os.path.join(ROOT, "profiles", "k_step_d3q27_f32_256cube.counters.json")


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(launch):
    """HBM bytes per launch of the FP32 step kernel from the committed
    rocprofv3 counter passes, if they were taken on these kernel sources and
    this launch shape; otherwise None."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("source_sha256") != kernel_source_hash() or list(c.get("launch", [])) != list(launch):
        return None
    return c["traffic_bytes_per_launch"]


REPEATS = 5  # further timed runs of `steps` steps, for the median


def time_steps(lat, steps, stream, torch):
    """Wall clock of `steps` steps on the lattice's stream (ms per step),
    bracketed by device synchronisations."""
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    lat.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


SETTLE_MS = 100.0  # GPU work queued right before every warm-up


def settle(scratch, est_ms_per_step, ms=SETTLE_MS):
    """Queue about `ms` milliseconds of steps of `scratch`, a lattice (or
    ensemble) of the same shape, storage and launch shape as the measured
    one but with buffers of its own, on the measured one's stream, without
    waiting for them.  The GPU lowers its clocks when it idles (a 2 s pause
    made the next 20 steps 11 % slower) and takes tens of milliseconds to
    raise them again; the warm-up steps queued behind this work then start
    at the clocks the step kernel itself sustains (after 100 ms of plain
    device copies instead, the first 20 timed steps behind a 5-step warm-up
    were 1.5 % slower than the later ones).  The measured lattice is not
    touched: it still takes exactly the requested warm-up steps."""
    scratch.step(max(2, int(ms / est_ms_per_step) + 1))


def est_ms(n_sites, storage, q=Q):
    """Rough step time for sizing the settle work: the algorithmic bytes at
    6 TB/s."""
    return n_sites * bytes_per_site(storage, q) / 6e9


def time_storage(storage, steps, warmup, stream, torch, tune=True, q=Q, in_place=False):
    from paper_2602_16486_amd import Lattice
    n = SHAPE[0] * SHAPE[1] * SHAPE[2]
    kw = dict(storage=storage, rho0=RHO0, tau=TAU, kT=KT, seed=SEED, stream=stream.cuda_stream,
              in_place=in_place)
    with Lattice(q, SHAPE, series_capacity=8192, **kw) as lat, \
            Lattice(q, SHAPE, series_capacity=64, **kw) as scratch:
        if tune:
            lat.autotune(steps_per_trial=10)  # untimed; state restored
        launch = lat.launch
        scratch.set_launch(*launch)
        settle(scratch, est_ms(n, storage, q))
        lat.step(warmup)
        # the headline: exactly `steps` steps after the warm-up
        ms_step = time_steps(lat, steps, stream, torch)
        repeats = [time_steps(lat, steps, stream, torch) for _ in range(REPEATS)]
        # live per-kernel duration of the fused step (HIP events around each
        # launch on the lattice's stream), same state, direct launches
        kprof = 20
        kernel_ms = lat.profile_steps(kprof) / kprof
        st = lat.stats()
    glups = n / (ms_step * 1e-3) / 1e9
    # equipartition over the recorded steps after the first 30 (warm-up)
    u2 = st[30:, 8:11].sum(axis=1) / (3 * n)
    return {
        "launch": launch,
        "ms_per_step": ms_step,
        "repeat_ms_per_step": repeats,
        "median_ms_per_step": float(sorted(repeats + [ms_step])[(REPEATS + 1) // 2]),
        "glups": glups,
        "kernel_ms": kernel_ms,
        "kernel_gbs": bytes_per_site(storage, q) * n / (kernel_ms * 1e-3) / 1e9,
        "u2_over_kT": float(u2.mean() * RHO0 / KT) if KT > 0 else None,
        "u2_series": u2,
        "nonfinite": float(st[:, 11].sum()),
    }


def ensemble_run(steps, warmup, stream, torch, eq_steps=1000, tune=True):
    """The mixed ensemble: 256 D2Q9 replicas (edges uniform in [32, 512] per axis) and
    64 D3Q27 replicas (edges uniform in [32, 96]), each with its own seed,
    kT log-uniform in [1e-6, 1e-3] and tau uniform in [0.502, 2.0], FP32,
    one launch per step; compared with the same replicas stepped one
    lattice at a time (same kernels, separate launches).  The tile shape is
    autotuned first (state restored by the tuner)."""
    import numpy as np
    from paper_2602_16486_amd import Ensemble, Lattice
    from paper_2602_16486_amd import workloads as W
    manifest = W.ensemble_manifest()
    total = sum(W.n_sites(r["shape"]) for r in manifest)
    with Ensemble(manifest, storage="f32", stream=stream.cuda_stream, series_capacity=4096) as ens:
        if tune:
            ens.autotune(steps_per_trial=4)
        tiles = ens.tiles
        # the scratch ensemble lives until the timed run is over (freeing it
        # in between would idle the GPU)
        with Ensemble(manifest, storage="f32", stream=stream.cuda_stream, series_capacity=64) as scratch:
            scratch.set_tiles(*tiles)
            settle(scratch, sum(est_ms(W.n_sites(r["shape"]), "f32", r["q"]) for r in manifest))
            ens.step(warmup)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ens.step(steps)
            b.record(stream)
            torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        kernel_ms = ens.profile_steps(10) / 10
        # equipartition per replica over the second half of eq_steps steps
        ens.step(eq_steps - (steps + warmup + 10) % eq_steps)
        ratios = []
        for k, r in enumerate(manifest):
            st = ens.stats(k)
            n = W.n_sites(r["shape"])
            half = st[len(st) // 2:]
            dims = 2 if r["q"] == 9 else 3
            ratios.append(float(half[:, 8:8 + dims].sum(axis=1).mean() / (dims * n) * r["rho0"] / r["kT"]))
    # time split by lattice type: the D2Q9 and the D3Q27 replicas of the
    # manifest as ensembles of their own, in the tile shape just used
    split = {}
    for q in (9, 27):
        part = [r for r in manifest if r["q"] == q]
        with Ensemble(part, storage="f32", stream=stream.cuda_stream, series_capacity=64) as sub:
            sub.set_tiles(*tiles)
            sub.step(4)
            split[f"d2q9_ms" if q == 9 else "d3q27_ms"] = sub.profile_steps(10) / 10
    # lanes the tiles leave idle: a tile is spt x 256 consecutive sites of
    # one replica, so only the last tile of a replica is ragged
    idle = {}
    for q in (9, 27):
        lanes = sites = 0
        for r in manifest:
            if r["q"] != q:
                continue
            tl = (tiles[0] if q == 9 else tiles[1]) * 256
            n = W.n_sites(r["shape"])
            lanes += -(-n // tl) * tl
            sites += n
        idle["d2q9" if q == 9 else "d3q27"] = 1.0 - sites / lanes
    # the same replicas one at a time
    seq_ms = 0.0
    nseq = 20
    for r in manifest:
        with Lattice(r["q"], r["shape"], storage="f32", tau=r["tau"], kT=r["kT"], seed=r["seed"],
                     replica=r["replica"], stream=stream.cuda_stream) as lat:
            lat.step(2)
            torch.cuda.synchronize()
            a.record(stream)
            lat.step(nseq)
            b.record(stream)
            torch.cuda.synchronize()
            seq_ms += a.elapsed_time(b) / nseq
    ratios = np.array(ratios)
    return {
        "value": total / (ms * 1e-3) / 1e9, "unit": "GLUPS", "ms_per_step": ms,
        "kernel_ms": kernel_ms, "sites": total, "replicas": len(manifest),
        "tiles_sites_per_thread": {"d2q9": tiles[0], "3d": tiles[1]},
        "bytes_per_step": sum(W.n_sites(r["shape"]) * 2 * r["q"] * 4 for r in manifest),
        "split_kernel_ms": split,
        "idle_lane_fraction": idle,
        "sequential_single_replica_glups": total / (seq_ms * 1e-3) / 1e9,
        "speedup_vs_sequential": seq_ms / ms,
        "u2_over_kT_median": float(np.median(ratios)),
        "u2_over_kT_p05_p95": [float(np.percentile(ratios, 5)), float(np.percentile(ratios, 95))],
        "equipartition_window": f"steps {eq_steps // 2}-{eq_steps}",
    }


def cpu_baseline():
    """The FP64 oracle, as it is, on the host cores: D3Q27 64^3 for 100 steps
    from rest (same parameters as the GPU workload) with the dense T(u) + LU
    reconstruction on every thread (the reported value), plus D2Q9 1024^2
    for 200 steps (the D2Q9 workload's box), the oracle's second
    reconstruction form (M^-1 N(-u), 64^3 x 40 steps) and both forms on one
    core (32^3 x 10 steps)."""
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))

    def timed(shape, steps, method, nthreads, q=Q):
        n = 1
        for e in shape:
            n *= e
        f = O.init_equilibrium(q, n, rho0=RHO0)
        t0 = time.perf_counter()
        O.run(q, shape, f, KT, O.paper_lambda(q, 1 / TAU), SEED, 0, 0, steps, method=method,
              nthreads=nthreads)
        dt = time.perf_counter() - t0
        return n * steps / dt, dt

    rate, dt = timed((64, 64, 64), 100, 0, threads)
    d2q9, dt9 = timed((1024, 1024), 200, 0, threads, q=9)
    shift, _ = timed((64, 64, 64), 40, 1, threads)
    one_lu, _ = timed((32, 32, 32), 10, 0, 1)
    one_shift, _ = timed((32, 32, 32), 10, 1, 1)
    return {"value": rate / 1e9, "unit": "GLUPS", "cores": threads, "kind": "oracle",
            "sample": f"D3Q27 64^3 x 100 steps from rest (rho0=1, tau=0.8, kT=1e-4, seed 1), "
                      f"FP64 dense T(u) + LU, {dt:.1f} s",
            "d2q9_1024": {"value": d2q9 / 1e9, "unit": "GLUPS",
                          "sample": f"D2Q9 1024^2 x 200 steps from rest, same parameters, FP64 "
                                    f"dense T(u) + LU, {dt9:.1f} s"},
            "forms_mlups": {"dense_lu": rate / 1e6, "shift_reconstruction": shift / 1e6,
                            "dense_lu_one_core": one_lu / 1e6,
                            "shift_reconstruction_one_core": one_shift / 1e6}}


def main():
    global KT
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--variants", default="f16,bf16")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--kT", type=float, default=KT,
                    help="thermal energy of the timed lattices (profiling aid: 0 switches the "
                         "noise off; the headline workload is 1e-4)")
    ap.add_argument("--d3q19", default="f32,f16",
                    help="storages of the D3Q19 256^3 lines (empty: none)")
    ap.add_argument("--in-place", default="f32",
                    help="storages of the D3Q27 256^3 lines with in-place (AA) streaming, one "
                         "population buffer (empty: none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    KT = args.kT
    if args.steps < 1 or args.warmup < 0:
        print("need --steps >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2602_16486_amd import _lib
    if _lib.device_count() < 1 or not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()  # default priority
    n = SHAPE[0] * SHAPE[1] * SHAPE[2]

    log(f"timing f32: {args.warmup} warm-up + {args.steps} timed steps")
    main_run = time_storage("f32", args.steps, args.warmup, stream, torch, tune=not args.no_tune)
    log(f"f32: {main_run['ms_per_step']:.4f} ms/step, {main_run['glups']:.2f} GLUPS")
    variants = {}
    for storage in [s for s in args.variants.split(",") if s]:
        log(f"timing {storage}")
        r = time_storage(storage, args.steps, args.warmup, stream, torch, tune=not args.no_tune)
        m = min(len(r["u2_series"]), len(main_run["u2_series"]))
        du = float(np.abs(r["u2_series"][:m].mean() / main_run["u2_series"][:m].mean() - 1))
        variants[storage] = {
            "value": r["glups"], "ms_per_step": r["ms_per_step"],
            "median_ms_per_step": r["median_ms_per_step"], "kernel_ms": r["kernel_ms"],
            "kernel_gbs": r["kernel_gbs"], "frac_hbm": r["kernel_gbs"] / PEAK_HBM_GBS,
            "launch": list(r["launch"]),
            "bytes_per_site": bytes_per_site(storage),
            "u2_over_kT": r["u2_over_kT"], "u2_rel_diff_vs_f32": du,
        }
        log(f"{storage}: {r['glups']:.2f} GLUPS, <u2> rel diff vs f32 {du:.2e}")

    lattices = {}
    for storage in [s for s in args.d3q19.split(",") if s]:
        log(f"timing D3Q19 {storage}")
        r = time_storage(storage, args.steps, args.warmup, stream, torch, tune=not args.no_tune, q=19)
        lattices[f"d3q19_{storage}"] = {
            "value": r["glups"], "ms_per_step": r["ms_per_step"],
            "median_ms_per_step": r["median_ms_per_step"], "kernel_ms": r["kernel_ms"],
            "kernel_gbs": r["kernel_gbs"], "frac_hbm": r["kernel_gbs"] / PEAK_HBM_GBS,
            "launch": list(r["launch"]), "bytes_per_site": bytes_per_site(storage, 19),
            "u2_over_kT": r["u2_over_kT"],
        }
        log(f"D3Q19 {storage}: {r['glups']:.2f} GLUPS, kernel {r['kernel_gbs']:.0f} GB/s")

    in_place = {}
    for storage in [s for s in args.in_place.split(",") if s]:
        log(f"timing in-place {storage}")
        r = time_storage(storage, args.steps, args.warmup, stream, torch, tune=not args.no_tune,
                         in_place=True)
        ref = main_run if storage == "f32" else None
        entry = {
            "value": r["glups"], "ms_per_step": r["ms_per_step"],
            "median_ms_per_step": r["median_ms_per_step"], "kernel_ms": r["kernel_ms"],
            "kernel_gbs": r["kernel_gbs"], "frac_hbm": r["kernel_gbs"] / PEAK_HBM_GBS,
            "launch": list(r["launch"]), "bytes_per_site": bytes_per_site(storage),
            "population_bytes": Q * n * {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[storage],
            "u2_over_kT": r["u2_over_kT"],
        }
        if ref is not None:
            m = min(len(r["u2_series"]), len(ref["u2_series"]))
            a, c = r["u2_series"][:m], ref["u2_series"][:m]
            entry["u2_rel_diff_vs_pull"] = float(np.abs(a - c).max() / np.abs(c).mean())
        in_place[storage] = entry
        log(f"in-place {storage}: {r['glups']:.2f} GLUPS, kernel {r['kernel_ms']:.4f} ms")

    copy_bytes = Q * n * 4  # one FP32 population buffer: the step's footprint
    copy_ms = _lib.stream_copy(copy_bytes, reps=5)
    copy_gbs = 2 * copy_bytes / (copy_ms * 1e-3) / 1e9
    log(f"plain copy of {copy_bytes / 1e9:.2f} GB: {copy_gbs:.0f} GB/s")
    achieved = main_run["kernel_gbs"]
    result = {
        "metric": "D3Q27 256^3 GLUPS (fused fluctuating CM step)",
        "value": main_run["glups"],
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"D3Q27 256^3 periodic, rest start, rho0=1, tau=0.8, kT={KT:g}, Philox seed 1; "
                        "FP32 deviation storage, FP32 collide, FP64 per-step statistics",
            "lattice": "D3Q27", "box": list(SHAPE), "storage": "f32",
            "bytes_per_site_step": bytes_per_site("f32"),
            "launch": list(main_run["launch"]),
            # environment variables that select launch or tile shapes (never results)
            "env": {k: os.environ[k] for k in ("CMFLB_TUNE_CACHE", "CMF_BLOCK", "CMF_GRID", "CMF_ENSEMBLE_SPT9",
                                               "CMF_ENSEMBLE_SPT27") if k in os.environ},
        },
        "timing": {
            "protocol": f"autotuning (state restored), about {SETTLE_MS:.0f} ms of steps of a scratch lattice of "
                        f"the same shape and launch shape (buffers of its own; clocks up, the measured lattice "
                        f"untouched) queued on the lattice's stream, {args.warmup} warm-up steps, "
                        f"then {args.steps} timed steps (the value); "
                        f"then {REPEATS} more timed runs of {args.steps} steps; CUDA/HIP events on "
                        f"the lattice's stream around cmf_step (32-step graph replays and direct "
                        f"steps, statistics reductions overlapped on a second stream)",
            "repeat_ms_per_step": main_run["repeat_ms_per_step"],
            "median_ms_per_step": main_run["median_ms_per_step"],
            "median_glups": n / (main_run["median_ms_per_step"] * 1e-3) / 1e9,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": measured_traffic(main_run["launch"]),
            "kernel_ms": main_run["kernel_ms"],
            "bytes_per_launch": bytes_per_site("f32") * n,
            "copy_ceiling_gbs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
        },
        "u2_over_kT": main_run["u2_over_kT"],
        "variants": variants,
        "lattices": lattices,
        "in_place": in_place,
    }
    if not args.no_ensemble:
        log("timing the batched ensemble (256 D2Q9 + 64 D3Q27 replicas)")
        ens = ensemble_run(min(args.steps, 200), 40, stream, torch, tune=not args.no_tune)
        ens["achieved_gbs"] = ens["bytes_per_step"] / (ens["kernel_ms"] * 1e-3) / 1e9
        result["ensemble"] = ens
        log(f"ensemble: {ens['value']:.2f} GLUPS ({ens['speedup_vs_sequential']:.2f}x the sequential runs)")
    if not args.no_cpu:
        log("timing the CPU oracle sample")
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
