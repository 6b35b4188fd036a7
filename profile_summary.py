#!/usr/bin/env python3
"""Summarise the rocprofv3 runs of bench.py into profiles/.

Inputs (written by rocprofv3 under a results directory, `out/` in the
commands below; any directory works):
  <dir>/prof_trace/trace_kernel_stats.csv        (--kernel-trace --stats)
  <dir>/prof_fetch/fetch_counter_collection.csv  (--pmc FETCH_SIZE)
  <dir>/prof_write/write_counter_collection.csv  (--pmc WRITE_SIZE)
  <dir>/prof_trace.json                          (bench.py's JSON line of the trace run)

The HBM byte counters are calibrated with the plain copy kernel that
bench.py runs (cmf_stream_copy_kernel, which reads and writes exactly
27 * 256^3 * 4 bytes): factor = known bytes / counter reading, per counter.

Outputs: profiles/k_step_d3q27_f32_256cube.md (the summary) and
profiles/k_step_d3q27_f32_256cube.counters.json (read by bench.py, tied to
the kernel sources' hash and the launch shape).

    python profile_summary.py out
"""
import csv
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
import bench  # noqa: E402  (kernel_source_hash, constants)

STEP_KERNEL = "void cmf::k_step<cmf::D3Q27, float, float, false, true, false, true>"
COPY_KERNEL = "cmf::cmf_stream_copy_kernel"
N = 256 ** 3
ALG_BYTES = 2 * 27 * 4 * N
COPY_BYTES = 27 * N * 4  # per direction

CMD_TRACE = ("rocprofv3 --kernel-trace --stats -d out/prof_trace -o trace --output-format csv "
             "-- python3 bench.py --steps 400 --warmup 64 --variants \"\" --d3q19 \"\" --in-place \"\" --no-cpu "
             "--no-tune --no-ensemble")
CMD_FETCH = ("rocprofv3 --pmc FETCH_SIZE -d out/prof_fetch -o fetch --output-format csv "
             "-- python3 bench.py --steps 10 --warmup 32 --variants \"\" --d3q19 \"\" --in-place \"\" --no-cpu "
             "--no-tune --no-ensemble")
CMD_WRITE = CMD_FETCH.replace("FETCH_SIZE", "WRITE_SIZE").replace("prof_fetch", "prof_write").replace(
    "-o fetch", "-o write")


def _median_counter(path, kernel):
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if r["Kernel_Name"].startswith(kernel)]
    return statistics.median(vals), len(vals)


def main(outdir):
    stats = {r["Name"]: r for r in csv.DictReader(open(os.path.join(outdir, "prof_trace", "trace_kernel_stats.csv")))}
    step = next(v for k, v in stats.items() if k.startswith(STEP_KERNEL))
    copy = next(v for k, v in stats.items() if k.startswith(COPY_KERNEL))
    fetch_step, nf = _median_counter(os.path.join(outdir, "prof_fetch", "fetch_counter_collection.csv"), STEP_KERNEL)
    fetch_copy, _ = _median_counter(os.path.join(outdir, "prof_fetch", "fetch_counter_collection.csv"), COPY_KERNEL)
    write_step, nw = _median_counter(os.path.join(outdir, "prof_write", "write_counter_collection.csv"), STEP_KERNEL)
    write_copy, _ = _median_counter(os.path.join(outdir, "prof_write", "write_counter_collection.csv"), COPY_KERNEL)
    bench_line = json.loads(open(os.path.join(outdir, "prof_trace.json")).read().strip().splitlines()[-1])
    launch = bench_line["config"]["launch"]
    f_fetch = COPY_BYTES / (fetch_copy * 1024)
    f_write = COPY_BYTES / (write_copy * 1024)
    read_b = fetch_step * 1024 * f_fetch
    write_b = write_step * 1024 * f_write
    traffic = read_b + write_b
    avg_ns = float(step["AverageNs"])
    durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            for r in csv.DictReader(open(os.path.join(outdir, "prof_trace", "trace_kernel_trace.csv")))
            if r["Kernel_Name"].startswith(STEP_KERNEL)]
    med_ns = statistics.median(durs)
    rec = {
        "kernel": STEP_KERNEL, "workload": bench_line["config"]["workload"], "launch": launch,
        "source_sha256": bench.kernel_source_hash(),
        "fetch_kib_per_dispatch": fetch_step, "write_kib_per_dispatch": write_step,
        "fetch_factor": f_fetch, "write_factor": f_write,
        "read_bytes_per_launch": read_b, "write_bytes_per_launch": write_b,
        "traffic_bytes_per_launch": traffic, "algorithmic_bytes_per_launch": ALG_BYTES,
        "traffic_over_algorithmic": traffic / ALG_BYTES,
        "rocprof_avg_ns": avg_ns, "rocprof_median_ns": med_ns,
        "bench_kernel_ms": bench_line["roofline"]["kernel_ms"],
    }
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "k_step_d3q27_f32_256cube.counters.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    lines = [
        "# k_step<D3Q27, f32> on D3Q27 256^3 (bench workload) — rocprofv3 summary",
        "",
        "Workload: " + bench_line["config"]["workload"] + f"; launch (block, grid) = {tuple(launch)}.",
        "",
        "Commands (run from the repository root on a machine with an MI355X, after `cd /tmp && export TMPDIR=/tmp`;",
        "the three runs share one tuning cache, `CMFLB_TUNE_CACHE=out/tune.txt`, written by a",
        "preceding `python bench.py`):",
        "",
        "    " + CMD_TRACE,
        "    " + CMD_FETCH,
        "    " + CMD_WRITE,
        "    python profile_summary.py out",
        "",
        "## Kernel trace (--kernel-trace --stats)",
        "",
        "| kernel | calls | average ns | min ns | max ns |",
        "|---|---|---|---|---|",
    ]
    for k, v in sorted(stats.items(), key=lambda kv: -float(kv[1]["TotalDurationNs"])):
        lines.append(f"| `{k[:90]}` | {v['Calls']} | {float(v['AverageNs']):.0f} | {v['MinNs']} | {v['MaxNs']} |")
    lines += [
        "",
        f"Step kernel: {avg_ns / 1e6:.4f} ms average, {med_ns / 1e6:.4f} ms median over {len(durs)} dispatches; "
        f"bench.py's live HIP-event measurement of the same kernel: {bench_line['roofline']['kernel_ms']:.4f} ms.",
        f"Achieved (algorithmic {ALG_BYTES} B per launch = 216 B/site x 256^3, median duration): "
        f"{ALG_BYTES / (med_ns * 1e-9) / 1e9:.0f} GB/s = {ALG_BYTES / (med_ns * 1e-9) / 8e12:.3f} of 8 TB/s.",
        f"Plain copy kernel: {float(copy['AverageNs']) / 1e6:.4f} ms for 2 x {COPY_BYTES} B = "
        f"{2 * COPY_BYTES / (float(copy['AverageNs']) * 1e-9) / 1e9:.0f} GB/s.",
        "",
        "## HBM bytes (--pmc FETCH_SIZE, then WRITE_SIZE; KiB per dispatch, median)",
        "",
        "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB |",
        "|---|---|---|",
        f"| step ({nf}/{nw} dispatches) | {fetch_step:.0f} | {write_step:.0f} |",
        f"| plain copy (known {COPY_BYTES // 1024} KiB each way) | {fetch_copy:.0f} | {write_copy:.0f} |",
        "",
        f"Calibration factors (known bytes / counter): FETCH x{f_fetch:.4f}, WRITE x{f_write:.4f}.",
        f"Step kernel traffic per launch: read {read_b / 1e9:.3f} GB + write {write_b / 1e9:.3f} GB = "
        f"{traffic / 1e9:.3f} GB, {traffic / ALG_BYTES:.3f} x the algorithmic {ALG_BYTES / 1e9:.3f} GB "
        f"(reads {read_b / (ALG_BYTES / 2):.3f} x, writes {write_b / (ALG_BYTES / 2):.3f} x).",
        "",
    ]
    with open(os.path.join(ROOT, "profiles", "k_step_d3q27_f32_256cube.md"), "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


ENS_KERNEL = "void cmf::k_ensemble_step<float, float, false>"
CMD_ENS = ("rocprofv3 --kernel-trace --stats -d out/prof_ens -o ens --output-format csv "
           "-- python3 bench.py --steps 50 --warmup 16 --variants \"\" --d3q19 \"\" --in-place \"\" --no-cpu "
           "--no-tune")
CMD_ENS_FETCH = ("rocprofv3 --pmc FETCH_SIZE -d out/prof_ens_fetch -o ens_fetch --output-format csv "
                 "-- python3 bench.py --steps 10 --warmup 8 --variants \"\" --d3q19 \"\" --in-place \"\" "
                 "--no-cpu --no-tune")
CMD_ENS_WRITE = CMD_ENS_FETCH.replace("FETCH_SIZE", "WRITE_SIZE").replace("ens_fetch", "ens_write")
CMD_ENS_VALU = CMD_ENS_FETCH.replace("FETCH_SIZE", "SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES "
                                     "SQ_WAVE_CYCLES SQ_INSTS_SALU SQ_ACTIVE_INST_ANY GRBM_GUI_ACTIVE").replace(
    "ens_fetch", "ens_valu")


def ensemble_summary(outdir):
    """profiles/k_ensemble_step_mixed320.md from the kernel trace of a bench
    run with the ensemble leg (prof_ens/, prof_ens.json)."""
    path = os.path.join(outdir, "prof_ens", "ens_kernel_stats.csv")
    if not os.path.exists(path):
        return
    stats = {r["Name"]: r for r in csv.DictReader(open(path))}
    ens = next(v for k, v in stats.items() if k.startswith(ENS_KERNEL))
    durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            for r in csv.DictReader(open(os.path.join(outdir, "prof_ens", "ens_kernel_trace.csv")))
            if r["Kernel_Name"].startswith(ENS_KERNEL)]
    line = json.loads(open(os.path.join(outdir, "prof_ens.json")).read().strip().splitlines()[-1])
    e = line["ensemble"]
    alg = e["bytes_per_step"]
    med = statistics.median(durs)
    lines = [
        "# k_ensemble_step<f32> on the mixed ensemble (256 D2Q9 + 64 D3Q27 replicas) — rocprofv3 summary",
        "",
        f"Workload: {e['replicas']} replicas, {e['sites']} sites, {alg} algorithmic bytes per step "
        "(2 Q 4 B per site, summed over the replicas).",
        "",
        f"Tile shape: {e['tiles_sites_per_thread']['d2q9']} (D2Q9) and {e['tiles_sites_per_thread']['3d']} (3-D) "
        "sites per thread, the shape `python bench.py` tuned, passed through the environment.",
        "",
        "Command (repository root on a machine with an MI355X, after `cd /tmp && export TMPDIR=/tmp`):",
        "",
        f"    export CMF_ENSEMBLE_SPT9={e['tiles_sites_per_thread']['d2q9']} "
        f"CMF_ENSEMBLE_SPT27={e['tiles_sites_per_thread']['3d']}",
        "    " + CMD_ENS,
        "    python profile_summary.py out",
        "",
        "| kernel | calls | average ns | min ns | max ns |",
        "|---|---|---|---|---|",
    ]
    for k, v in sorted(stats.items(), key=lambda kv: -float(kv[1]["TotalDurationNs"]))[:12]:
        lines.append(f"| `{k[:90]}` | {v['Calls']} | {float(v['AverageNs']):.0f} | {v['MinNs']} | {v['MaxNs']} |")
    lines += [
        "",
        f"Ensemble step kernel: {float(ens['AverageNs']) / 1e6:.4f} ms average, {med / 1e6:.4f} ms median over "
        f"{len(durs)} dispatches (bench.py's HIP-event figure: {e['kernel_ms']:.4f} ms); "
        f"{alg / (med * 1e-9) / 1e9:.0f} GB/s algorithmic = {alg / (med * 1e-9) / 8e12:.3f} of 8 TB/s, "
        f"{e['sites'] / (med * 1e-9) / 1e9:.1f} GLUPS.",
        f"Time split (one launch over the D2Q9 replicas only, one over the D3Q27 replicas only, same tiles): "
        f"{e['split_kernel_ms']['d2q9_ms']:.4f} / {e['split_kernel_ms']['d3q27_ms']:.4f} ms; idle lanes "
        f"{e['idle_lane_fraction']['d2q9'] * 100:.2f} % / {e['idle_lane_fraction']['d3q27'] * 100:.2f} %.",
        "",
    ]
    fpath = os.path.join(outdir, "prof_ens_fetch", "ens_fetch_counter_collection.csv")
    wpath = os.path.join(outdir, "prof_ens_write", "ens_write_counter_collection.csv")
    if os.path.exists(fpath) and os.path.exists(wpath):
        fe, nf = _median_counter(fpath, ENS_KERNEL)
        fc, _ = _median_counter(fpath, COPY_KERNEL)
        we, nw = _median_counter(wpath, ENS_KERNEL)
        wc, _ = _median_counter(wpath, COPY_KERNEL)
        rb, wb = fe * 1024 * COPY_BYTES / (fc * 1024), we * 1024 * COPY_BYTES / (wc * 1024)
        lines += [
            "HBM bytes (same environment, calibrated by the plain copy kernel of the same runs as for the step "
            "kernel):",
            "",
            "    " + CMD_ENS_FETCH,
            "    " + CMD_ENS_WRITE,
            "",
            f"Ensemble kernel ({nf}/{nw} dispatches, medians): FETCH_SIZE {fe:.0f} KiB, WRITE_SIZE {we:.0f} KiB; "
            f"read {rb / 1e9:.3f} GB + write {wb / 1e9:.3f} GB = {(rb + wb) / 1e9:.3f} GB per launch, "
            f"{(rb + wb) / alg:.3f} x the algorithmic {alg / 1e9:.3f} GB (reads {rb / (alg / 2):.3f} x, "
            f"writes {wb / (alg / 2):.3f} x).",
            "",
        ]
    vpath = os.path.join(outdir, "prof_ens_valu", "ens_valu_counter_collection.csv")
    if os.path.exists(vpath):
        c = {}
        for r in csv.DictReader(open(vpath)):
            if r["Kernel_Name"].startswith(ENS_KERNEL):
                c.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        med = {k: statistics.median(v) for k, v in c.items()}
        per_xcd = med["GRBM_GUI_ACTIVE"] / XCC_NUM
        lines += [
            "Vector-ALU activity (one counter pass, medians over the ensemble kernel's dispatches; definitions as "
            "in `k_step_valu_256cube.md`):",
            "",
            "    " + CMD_ENS_VALU,
            "",
            f"VALU instructions per site (SQ_INSTS_VALU x 64 / sites, idle lanes included) "
            f"{med['SQ_INSTS_VALU'] * 64 / e['sites']:.0f}; quad-cycles per VALU instruction "
            f"{med['SQ_ACTIVE_INST_VALU'] / med['SQ_INSTS_VALU']:.3f}; VALU busy "
            f"{100 * med['SQ_ACTIVE_INST_VALU'] / CU_NUM / per_xcd:.0f} %.",
            "",
        ]
    with open(os.path.join(ROOT, "profiles", "k_ensemble_step_mixed320.md"), "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


CMD_VAR = ("rocprofv3 --kernel-trace --stats -d out/prof_var -o var --output-format csv "
           "-- python3 bench.py --steps 100 --warmup 32 --no-cpu --no-tune --no-ensemble")
VARIANTS = [  # (kernel name prefix, label, q, bytes per stored value, bench.py entry)
    ("void cmf::k_step<cmf::D3Q27, float, float, false, true, false, true>", "D3Q27 FP32", 27, 4, None),
    ("void cmf::k_step<cmf::D3Q27, __half, float, false, true, false, true>", "D3Q27 FP16", 27, 2, ("variants", "f16")),
    ("void cmf::k_step<cmf::D3Q27, __hip_bfloat16, float, false, true, false, true>", "D3Q27 BF16", 27, 2,
     ("variants", "bf16")),
    ("void cmf::k_step<cmf::D3Q19, float, float, false, true, false, true>", "D3Q19 FP32", 19, 4, ("lattices", "d3q19_f32")),
    ("void cmf::k_step<cmf::D3Q19, __half, float, false, true, false, true>", "D3Q19 FP16", 19, 2, ("lattices", "d3q19_f16")),
    ("void cmf::k_step_aa<cmf::D3Q27, float, float, false, true, false, false>", "D3Q27 FP32 in place, even step", 27, 4,
     ("in_place", "f32")),
    ("void cmf::k_step_aa<cmf::D3Q27, float, float, false, true, false, true>", "D3Q27 FP32 in place, odd step", 27, 4,
     ("in_place", "f32")),
]


CMD_IP_FETCH = ("rocprofv3 --pmc FETCH_SIZE -d out/prof_ip_fetch -o ip_fetch --output-format csv "
                "-- python3 bench.py --steps 10 --warmup 8 --variants \"\" --d3q19 \"\" --no-cpu --no-tune "
                "--no-ensemble")
CMD_IP_WRITE = CMD_IP_FETCH.replace("FETCH_SIZE", "WRITE_SIZE").replace("ip_fetch", "ip_write")


def variants_summary(outdir):
    """profiles/k_step_variants_256cube.md: every step-kernel instantiation
    the default bench run times at 256^3 (storage variants, D3Q19), from
    one kernel trace of that run."""
    path = os.path.join(outdir, "prof_var", "var_kernel_trace.csv")
    if not os.path.exists(path):
        return
    rows = list(csv.DictReader(open(path)))
    line = json.loads(open(os.path.join(outdir, "prof_var.json")).read().strip().splitlines()[-1])
    lines = [
        "# k_step instantiations at 256^3 (bench workload and its variants) — rocprofv3 summary",
        "",
        "Workload: 256^3 periodic, rest start, rho0=1, tau=0.8, kT=1e-4, Philox seed 1, the paper's rates; "
        "launch shapes from the tuning cache of a preceding `python bench.py` (`CMFLB_TUNE_CACHE`).",
        "",
        "Command (repository root on a machine with an MI355X, after `cd /tmp && export TMPDIR=/tmp`):",
        "",
        "    " + CMD_VAR,
        "    python profile_summary.py out",
        "",
        "| kernel | dispatches | average ms | median ms | bench.py live ms | algorithmic B/site | GB/s (median) | of 8 TB/s |",
        "|---|---|---|---|---|---|---|---|",
    ]
    for prefix, label, q, sbytes, entry in VARIANTS:
        durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows
                if r["Kernel_Name"].startswith(prefix)]
        if not durs:
            continue
        if entry is None:
            live = line["roofline"]["kernel_ms"]
        else:
            e = line.get(entry[0], {}).get(entry[1])
            if e is None:
                live = float("nan")
            elif "kernel_ms" in e:
                live = e["kernel_ms"]
            else:
                live = 2 * q * sbytes * N / (e["kernel_gbs"] * 1e9) * 1e3
        alg = 2 * q * sbytes * N
        med = statistics.median(durs)
        avg = sum(durs) / len(durs)
        lines.append(f"| {label} `{prefix[10:]}` | {len(durs)} | {avg / 1e6:.4f} | {med / 1e6:.4f} | {live:.4f} | "
                     f"{2 * q * sbytes} | {alg / (med * 1e-9) / 1e9:.0f} | {alg / (med * 1e-9) / 8e12:.3f} |")
    fpath = os.path.join(outdir, "prof_ip_fetch", "ip_fetch_counter_collection.csv")
    wpath = os.path.join(outdir, "prof_ip_write", "ip_write_counter_collection.csv")
    if os.path.exists(fpath) and os.path.exists(wpath):
        fc, _ = _median_counter(fpath, COPY_KERNEL)
        wc, _ = _median_counter(wpath, COPY_KERNEL)
        lines += ["", "HBM bytes of the FP32 pull and in-place kernels (FETCH_SIZE, then WRITE_SIZE, calibrated by the "
                  "plain copy kernel of the same runs):", "", "    " + CMD_IP_FETCH, "    " + CMD_IP_WRITE, "",
                  "| kernel | dispatches | read GB | write GB | traffic / algorithmic |", "|---|---|---|---|---|"]
        alg = 2 * 27 * 4 * N
        for prefix, label in ((STEP_KERNEL, "D3Q27 FP32 pull"), (VARIANTS[-2][0], VARIANTS[-2][1]),
                              (VARIANTS[-1][0], VARIANTS[-1][1])):
            fk, nf = _median_counter(fpath, prefix)
            wk, _ = _median_counter(wpath, prefix)
            rb, wb = fk * COPY_BYTES / fc, wk * COPY_BYTES / wc
            lines.append(f"| {label} | {nf} | {rb / 1e9:.3f} | {wb / 1e9:.3f} | {(rb + wb) / alg:.3f} |")
    lines += ["", "The 16-bit kernels are bound by instruction issue (the Philox4x32-10 and Box-Muller noise is "
              "about two thirds of it), not by HBM.  The in-place (AA) pair streams the same bytes in one buffer; "
              "bench.py's live figure for it is the average over even and odd steps.", ""]
    with open(os.path.join(ROOT, "profiles", "k_step_variants_256cube.md"), "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


VALU_COUNTERS = ("SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_SALU "
                 "SQ_ACTIVE_INST_ANY GRBM_GUI_ACTIVE")
CMD_VALU = ("CMFLB_TUNE_CACHE=out/tune.txt rocprofv3 --pmc " + VALU_COUNTERS + " -d out/prof_valu -o valu --output-format csv "
            "-- python3 bench.py --steps 10 --warmup 8 --in-place \"\" --no-cpu --no-tune --no-ensemble")
CU_NUM = 256
XCC_NUM = 8


def valu_summary(outdir):
    """profiles/k_step_valu_256cube.md: vector-ALU activity of every step
    kernel at 256^3 from one counter pass.  VALU busy is rocprofv3's VALUBusy,
    100 sum(SQ_ACTIVE_INST_VALU) / CU_NUM / max(GRBM_GUI_ACTIVE), where
    SQ_ACTIVE_INST_VALU counts quad-cycles (one wave64 instruction on a
    16-lane SIMD) summed over all SIMDs, and the per-dispatch
    GRBM_GUI_ACTIVE reading is the sum over the 8 XCDs (max = sum / 8)."""
    path = os.path.join(outdir, "prof_valu", "valu_counter_collection.csv")
    if not os.path.exists(path):
        return
    vals = {}
    launch = {}
    for r in csv.DictReader(open(path)):
        for prefix, label, q, sbytes, _ in VARIANTS:
            if r["Kernel_Name"].startswith(prefix):
                vals.setdefault(label, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
                launch[label] = (int(r["Workgroup_Size"]), int(r["Grid_Size"]) // int(r["Workgroup_Size"]))
    lines = [
        "# k_step vector-ALU activity at 256^3 — rocprofv3 counter summary",
        "",
        "Workload: as in `k_step_variants_256cube.md` (256^3, rest start, rho0=1, tau=0.8, kT=1e-4, "
        "Philox seed 1); launch shapes from the tuning cache of a preceding `python bench.py --no-cpu "
        "--no-ensemble` run (`CMFLB_TUNE_CACHE` set for both).",
        "",
        "Command (repository root on a machine with an MI355X, after `cd /tmp && export TMPDIR=/tmp`):",
        "",
        "    CMFLB_TUNE_CACHE=out/tune.txt python3 bench.py --no-cpu --no-ensemble > out/tune_run.json",
        "    " + CMD_VALU,
        "    python profile_summary.py out",
        "",
        "Medians over all dispatches of each kernel.  VALU instructions per site = SQ_INSTS_VALU x 64 / 256^3 "
        "(each wave instruction serves 64 sites); quad-cycles per instruction = SQ_ACTIVE_INST_VALU / "
        "SQ_INSTS_VALU (1 = a full-rate wave64 instruction); VALU busy = rocprofv3's VALUBusy, "
        "100 sum(SQ_ACTIVE_INST_VALU) / 256 CUs / max(GRBM_GUI_ACTIVE), with the per-dispatch GRBM_GUI_ACTIVE "
        "summed over the 8 XCDs (max = sum / 8).",
        "",
        "| kernel | launch (block, grid) | VALU instr / site | SALU instr / wave (64 sites) | quad-cycles / VALU instr | "
        "GPU cycles (per XCD) | VALU busy |",
        "|---|---|---|---|---|---|---|",
    ]
    for prefix, label, q, sbytes, _ in VARIANTS:
        c = vals.get(label)
        if not c:
            continue
        med = {k: statistics.median(v) for k, v in c.items()}
        per_xcd = med["GRBM_GUI_ACTIVE"] / XCC_NUM
        busy = 100 * med["SQ_ACTIVE_INST_VALU"] / CU_NUM / per_xcd
        lines.append(f"| {label} | {launch[label]} | {med['SQ_INSTS_VALU'] * 64 / N:.0f} | "
                     f"{med['SQ_INSTS_SALU'] * 64 / N:.0f} | "
                     f"{med['SQ_ACTIVE_INST_VALU'] / med['SQ_INSTS_VALU']:.3f} | {per_xcd:.4g} | {busy:.0f} % |")
    lines += ["", "About 100 % VALU busy means the vector ALUs issue every cycle: the 16-bit kernels are bound by "
              "instruction issue (noise generation and the FP32 collision), the FP32 kernels by HBM.", ""]
    with open(os.path.join(ROOT, "profiles", "k_step_valu_256cube.md"), "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


CMD_VALU0 = CMD_VALU.replace("prof_valu", "prof_valu0").replace("-o valu", "-o valu0").replace(
    "--no-ensemble", "--no-ensemble --kT 0")
CMD_ASM = ("/opt/rocm/lib/llvm/bin/clang++ -x hip --offload-arch=gfx950 --offload-device-only -O3 -std=c++17 "
           "-ffp-contract=on -I include -Xclang -target-feature -Xclang -packed-fp32-ops -S "
           "paper_2602_16486_amd/csrc/cmflb_step_pull.hip -o out/kernels.s")
# opcode classes of the static budget
CLASSES = [
    ("Philox4x32-10 (64-bit products, 3-input xor)", ("v_mad_u64_u32", "v_bitop3_b32")),
    ("Box-Muller (log2, sqrt, sin, cos; word to float)", ("v_log_f32", "v_sqrt_f32", "v_sin_f32", "v_cos_f32",
                                                           "v_cvt_f32_u32", "v_lshrrev_b32")),
    ("16-bit loads and stores (scale and convert)", ("v_fma_mix_f32", "v_fma_mixlo_f16", "v_cvt_pk_bf16_f32")),
    ("statistics (FP64 accumulation)", ("v_add_f64", "v_cvt_f64_f32")),
]


def _kernel_ops(asm_path, mangled_prefix):
    """Opcode counts of one kernel function in the assembly listing."""
    import collections
    lines = open(asm_path).read().split("\n")
    start = next(i for i, l in enumerate(lines) if l.startswith(mangled_prefix) and l.rstrip().endswith(":")
                 or (l.startswith(mangled_prefix) and ": " in l))
    end = next(i for i in range(start + 1, len(lines)) if lines[i].strip().startswith(".Lfunc_end"))
    ops = collections.Counter()
    for l in lines[start + 1:end]:
        t = l.strip()
        if not t or t.startswith((".", ";")) or t.endswith(":"):
            continue
        ops[t.split()[0].split("_e32")[0].split("_e64")[0]] += 1
    return ops


BUDGET_KERNELS = [  # (label, mangled-name prefix, counter label in VARIANTS)
    ("D3Q27 FP16", "_ZN3cmf6k_stepINS_5D3Q27E6__halffLb0ELb1ELb0ELb1E", "D3Q27 FP16"),
    ("D3Q27 BF16", "_ZN3cmf6k_stepINS_5D3Q27E14__hip_bfloat16fLb0ELb1ELb0ELb1E", "D3Q27 BF16"),
    ("D3Q27 FP32", "_ZN3cmf6k_stepINS_5D3Q27EffLb0ELb1ELb0ELb1E", "D3Q27 FP32"),
]


def _valu_per_site(path):
    vals = {}
    for r in csv.DictReader(open(path)):
        for prefix, label, q, sbytes, _ in VARIANTS:
            if r["Kernel_Name"].startswith(prefix) and r["Counter_Name"] == "SQ_INSTS_VALU":
                vals.setdefault(label, []).append(float(r["Counter_Value"]))
    return {k: statistics.median(v) * 64 / N for k, v in vals.items()}


def valu_budget(outdir):
    """profiles/k_step_valu_budget_256cube.md: VALU instructions per site of
    the step kernels with the noise on (kT = 1e-4) and off (kT = 0), measured,
    and the static instruction mix of each kernel by class."""
    on_path = os.path.join(outdir, "prof_valu", "valu_counter_collection.csv")
    off_path = os.path.join(outdir, "prof_valu0", "valu0_counter_collection.csv")
    asm = os.path.join(outdir, "kernels.s")
    if not (os.path.exists(on_path) and os.path.exists(off_path) and os.path.exists(asm)):
        return
    on, off = _valu_per_site(on_path), _valu_per_site(off_path)
    lines = [
        "# VALU budget per site of the step kernels at 256^3 — rocprofv3 counters and static instruction mix",
        "",
        "Workload: as in `k_step_valu_256cube.md` (D3Q27 and D3Q19 256^3, rest start, rho0=1, tau=0.8, "
        "Philox seed 1), once with kT = 1e-4 (the benchmark) and once with kT = 0 (noise off: the kernels "
        "skip the normals, everything else is the same work).",
        "",
        "Commands (repository root on a machine with an MI355X, after `cd /tmp && export TMPDIR=/tmp`; "
        "the assembly listing needs no GPU):",
        "",
        "    CMFLB_TUNE_CACHE=out/tune.txt python3 bench.py --no-cpu --no-ensemble > out/tune_run.json",
        "    " + CMD_VALU,
        "    " + CMD_VALU0,
        "    " + CMD_ASM,
        "    python profile_summary.py out",
        "",
        "## Measured (SQ_INSTS_VALU x 64 / 256^3, median over dispatches)",
        "",
        "| kernel | VALU instr / site, kT = 1e-4 | kT = 0 | noise (difference) |",
        "|---|---|---|---|",
    ]
    for _, label, _, _, _ in VARIANTS:
        if label in on and label in off:
            lines.append(f"| {label} | {on[label]:.0f} | {off[label]:.0f} | {on[label] - off[label]:.0f} "
                         f"({(on[label] - off[label]) / on[label] * 100:.0f} %) |")
    lines += ["", "## Static instruction mix of each kernel function (gfx950 assembly of the sources)", "",
              "Whole function: the per-tile loop body plus a prologue and the block reduction of the "
              "statistics at the end (a few percent); the 16-bit and FP32 step kernels run 8 and 1 tiles per "
              "workgroup in the benchmark's launch shapes.", ""]
    head = "| class | " + " | ".join(k[0] for k in BUDGET_KERNELS) + " |"
    lines += [head, "|---|" + "---|" * len(BUDGET_KERNELS)]
    counts = [_kernel_ops(asm, k[1]) for k in BUDGET_KERNELS]
    totals = [sum(v for o, v in c.items() if o.startswith("v_")) for c in counts]
    used = [0] * len(counts)
    for name, ops in CLASSES:
        row = []
        for j, c in enumerate(counts):
            n = sum(c.get(o, 0) for o in ops)
            used[j] += n
            row.append(str(n))
        lines.append(f"| {name} | " + " | ".join(row) + " |")
    lines.append("| collision, moments, addresses and the rest | " +
                 " | ".join(str(t - u) for t, u in zip(totals, used)) + " |")
    lines.append("| all VALU instructions | " + " | ".join(str(t) for t in totals) + " |")
    lines += ["", "Philox4x32-10 needs 10 rounds of two 32 x 32 -> 64-bit products per block and six blocks "
              "per D3Q27 site (the first round's products are shared between the blocks); the Box-Muller "
              "transform takes four hardware transcendentals per pair of normals.  Both are fixed by the noise "
              "definition, so the 16-bit kernels, which issue a VALU instruction every cycle, are bound by them.",
              ""]
    with open(os.path.join(ROOT, "profiles", "k_step_valu_budget_256cube.md"), "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "out")
    ensemble_summary(sys.argv[1] if len(sys.argv) > 1 else "out")
    variants_summary(sys.argv[1] if len(sys.argv) > 1 else "out")
    valu_summary(sys.argv[1] if len(sys.argv) > 1 else "out")
    valu_budget(sys.argv[1] if len(sys.argv) > 1 else "out")
