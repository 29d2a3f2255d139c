"""Throughput benchmark: FP64 particle-steps per second on one MI355X.

One benchmark step is one whole run of the 100,000-particle, four-giant-planet
workload (dt = 120 d, 1e6 steps by default): planet map, particle kernel and
compaction, with all inputs already resident in HBM (every step gets its own
simulation object, loaded before the timed region).  The scatter of the
results back to caller order (a few microseconds) runs when they are read,
after the timed region.

Prints one JSON line with the throughput (active particle-steps / wall time of
the timed steps), the roofline of the particle kernel (FP64 ALU bound; HIP
events around every particle launch), the executed FP64 fraction of peak from
the committed counter runs, and the CPU oracle's rate on a bounded sample of
the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 flops of one active particle-step at four planets and the
# method's five Newton steps: the oracle's step tallied on a counting number
# type (oracle.count_ops), weighted add = mul = 1, reciprocal 9, square root
# 12, sine-cosine pair 39 (oracle.OP_WEIGHTS); pinned by
# tests/test_oracle_pins.py::test_operation_count_per_planet_and_newton_step.
# The kernel executes fewer (its Newton loop stops once converged, its kick
# uses one reciprocal square root per planet); what it executes comes from the
# counter runs below and is reported as `executed_fp64`.
ALGORITHMIC_FLOPS_PER_PARTICLE_STEP = {4: 718}
# The paper's own CPU-vs-GPU figure, quoted with the hardware it names (sec. 1
# and sec. 5): GLISSE on a Tesla K20m ran about 100 times faster than the same
# integration on a CPU core it does not name.
PAPER_SPEEDUP = {"value": 100, "gpu": "NVIDIA Tesla K20m", "cpu": "unnamed CPU",
                 "where": "sec. 1 and sec. 5"}
FP64_PEAK_TFLOPS = 78.6
COUNTERS_JSON = os.path.join(ROOT, "profiles", "particle_queue_giants_100k_counters.json")
COUNTERS_MD = os.path.join(ROOT, "profiles", "particle_queue_giants_100k_counters.md")
PMC_PASSES = {
    "p1": "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 "
          "SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VALU_FLOPS_FP64_TRANS",
    "p2": "SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_ANY SQ_WAIT_INST_ANY "
          "SQ_WAIT_ANY SQ_INSTS_SALU SQ_INSTS_SMEM",
    "p3": "FETCH_SIZE",
    "p4": "WRITE_SIZE",
}
PMC_BENCH_ARGS = ("--nsteps 20000 --steps 1 --warmup 0 --no-cpu --no-adjoint --no-batched "
                  "--no-resonant --no-handoff --copy-calibration-mb 256")
# The resonant workload's counter pass: a 1,024-particle headline run (another
# kernel variant, left out) and 20,000 steps of the resonant workload.
RES_COUNTERS_JSON = os.path.join(ROOT, "profiles", "particle_queue_resonant_200k_counters.json")
RES_COUNTERS_MD = os.path.join(ROOT, "profiles", "particle_queue_resonant_200k_counters.md")
RES_PMC = ("SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 "
           "SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VALU_FLOPS_FP64")
RES_PMC_BENCH_ARGS = ("--nsteps 1024 --n 1024 --steps 1 --warmup 0 --no-cpu --no-adjoint "
                      "--no-batched --no-handoff --resonant-steps 20000")


def kernel_source_hash() -> str:
    """Fingerprint of the HIP sources' code (counter figures apply to one
    version): comments and whitespace are left out, so that only a change of
    the code itself invalidates them."""
    import hashlib
    import re
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2011_03484_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".h")):
            text = open(os.path.join(csrc, f)).read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            h.update(f.encode() + b"\0" + " ".join(text.split()).encode())
    return h.hexdigest()


def counter_figures(path: str = COUNTERS_JSON):
    """Per active particle-step figures of the committed counter runs (executed
    FP64 flops; calibrated HBM bytes), or None unless they were taken on the
    current kernel sources."""
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    return d if d.get("source_hash") == kernel_source_hash() else None


# the library's defaults (include/tpmvs.h): chunk length, first-chunk cap when
# the planet map runs alongside, work items per tile and chunk
DEFAULT_CHUNK_STEPS, FIRST_CHUNK_STEPS, DEFAULT_SUB_CHUNKS = 8192, 1024, 64


def default_chunks(nsteps: int) -> list:
    """Chunk lengths of an on-the-fly run of nsteps with the default options."""
    out, done = [], 0
    while done < nsteps:
        k = min(FIRST_CHUNK_STEPS if not out else DEFAULT_CHUNK_STEPS, nsteps - done)
        out.append(k)
        done += k
    return out


def summarize_counters(pmc_dir: str) -> None:
    """Write the counter summary (markdown) and its per-particle-step figures
    (json) from the four rocprofv3 --pmc passes under pmc_dir/p1..p4, each made
    by `rocprofv3 --pmc <PMC_PASSES[p]> --kernel-trace -f csv -d <pmc_dir>/<p>
    -o run -- python3 bench.py <PMC_BENCH_ARGS>` with its output in
    <pmc_dir>/<p>.log."""
    import collections
    import csv

    def label(r):
        k = r["Kernel_Name"]
        if "particle_queue" in k:
            return "particle_queue<4,5>"
        if "ephemeris_chunk" in k:
            return "ephemeris_chunk<4>"
        if "copyBuffer" in k and int(r["Grid_Size"]) == 131072:
            return "device copy 256 MiB"
        return None

    tot = collections.defaultdict(float)
    cnt = collections.Counter()
    for p in PMC_PASSES:
        for r in csv.DictReader(open(os.path.join(pmc_dir, p, "run_counter_collection.csv"))):
            lab = label(r)
            if lab:
                tot[(p, lab, r["Counter_Name"])] += float(r["Counter_Value"])
                cnt[(p, lab, r["Counter_Name"])] += 1
    kt, kn = 0.0, 0
    for r in csv.DictReader(open(os.path.join(pmc_dir, "p2", "run_kernel_trace.csv"))):
        if "particle_queue" in r["Kernel_Name"]:
            kt += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
            kn += 1
    runs = {p: json.loads([x for x in open(os.path.join(pmc_dir, p + ".log")) if x.startswith("{")][-1])
            for p in PMC_PASSES}
    src = {r["kernel_sources"] for r in runs.values()}
    if len(src) != 1:
        raise SystemExit(f"counter passes ran on different kernel sources: {src}")
    src = src.pop()
    aps = runs["p1"]["active_particle_steps"]
    pq = "particle_queue<4,5>"
    g = lambda p, c, lab=pq: tot[(p, lab, c)]
    launches = cnt[("p1", pq, "SQ_WAVES")]
    waves = g("p1", "SQ_WAVES") / launches
    fetch_f = 262144.0 / g("p3", "FETCH_SIZE", "device copy 256 MiB")
    write_f = 262144.0 / g("p4", "WRITE_SIZE", "device copy 256 MiB")
    fetch_b = g("p3", "FETCH_SIZE") / launches * 1024 * fetch_f
    write_b = g("p4", "WRITE_SIZE") / launches * 1024 * write_f
    bpps = (fetch_b + write_b) / (aps / launches)
    per = lambda c: 64 * g("p1", c) / aps
    fpps = per("SQ_INSTS_VALU_FLOPS_FP64")
    steps = int(PMC_BENCH_ARGS.split()[1])
    chunks = default_chunks(steps)
    item = DEFAULT_CHUNK_STEPS // DEFAULT_SUB_CHUNKS
    items = [-(-k // item) for k in chunks]
    alg_b = 100.0 * sum(items) / steps
    out = [f"# particle_queue<4,5> counters -- giants_100k, 100,000 particles x {steps:,} steps "
           f"({launches} launches)", "",
           "Commands (one rocprofv3 run per pass, `cd /tmp && export TMPDIR=/tmp` first), then "
           "`python3 bench.py --summarize-counters <out>` for this summary:", ""]
    for p, c in PMC_PASSES.items():
        out.append(f"    timeout -s KILL 90 rocprofv3 --pmc {c} --kernel-trace -f csv -d <out>/{p} "
                   f"-o run -- python3 <repo>/bench.py {PMC_BENCH_ARGS} > <out>/{p}.log")
    out += ["", f"Kernel sources of the counted runs: `bench.kernel_source_hash()` = `{src}`.", "",
            f"Sums over the {launches} dispatches of the particle kernel and over the one 256 MiB "
            "device-to-device copy (its source evicted from the last-level cache first by writing "
            "a 1 GiB buffer), from `run_counter_collection.csv`:", "",
            "| kernel | counter | value |", "|---|---|---|"]
    for (p, lab, c), v in tot.items():
        out.append(f"| {lab} | {c} | {v:.6g} |")
    busy = g("p2", "SQ_ACTIVE_INST_VALU") / (1024 * kt * 2.4e9 / 4)
    out += ["", f"Derived (particle kernel; kernel-trace time of pass 2 = {kt * 1e3:.1f} ms for "
                f"{kn} launches; {aps:,} active particle-steps):", "",
            f"* VALU instructions per wavefront-step: {g('p1', 'SQ_INSTS_VALU'):.4g} / ({waves:.0f} "
            f"waves x {steps:,} steps) = {g('p1', 'SQ_INSTS_VALU') / (waves * steps):.0f}.",
            f"* Executed FP64 per active particle-step (64 x instructions / particle-steps): "
            f"{per('SQ_INSTS_VALU_FMA_F64'):.1f} FMA, {per('SQ_INSTS_VALU_MUL_F64'):.1f} mul, "
            f"{per('SQ_INSTS_VALU_ADD_F64'):.1f} add, {per('SQ_INSTS_VALU_TRANS_F64'):.1f} "
            f"transcendental; flops (FMA = 2) {fpps:.1f}.  The method's five Newton steps count "
            f"{ALGORITHMIC_FLOPS_PER_PARTICLE_STEP[4]} (the algorithmic figure of the roofline); "
            "lanes stop once converged.  Masked lanes of removed particles are included.",
            f"* SIMD VALU occupancy: SQ_ACTIVE_INST_VALU / (1024 SIMDs x {kt * 1e3:.1f} ms x 2.4 GHz "
            f"/ 4) = {busy * 100:.0f}%.",
            f"* FP64 rate under the profiler: {fpps:.1f} x {aps:.4g} / {kt * 1e3:.1f} ms = "
            f"{fpps * aps / kt / 1e12:.1f} TFLOP/s = {fpps * aps / kt / 1e12 / FP64_PEAK_TFLOPS * 100:.0f}% "
            f"of {FP64_PEAK_TFLOPS}.",
            f"* Calibration: the 256 MiB copy reads FETCH_SIZE "
            f"{g('p3', 'FETCH_SIZE', 'device copy 256 MiB'):.0f} KiB (factor {fetch_f:.4f}) and "
            f"WRITE_SIZE {g('p4', 'WRITE_SIZE', 'device copy 256 MiB'):.0f} KiB (factor {write_f:.4f}).",
            f"* HBM traffic per launch, calibrated: fetch {fetch_b / 1e6:.2f} MB + write "
            f"{write_b / 1e6:.2f} MB = {(fetch_b + write_b) / 1e6:.2f} MB for {aps / launches:,.0f} "
            f"active particle-steps, i.e. {bpps:.4f} B per particle-step (algorithmic: each "
            f"particle's state, 52 B in and 48 B out, moves once per work item of {item} steps; with the "
            f"library's default layout this run has chunks of {', '.join(f'{k:,}' for k in chunks)} "
            f"steps with {', '.join(str(i) for i in items)} items, so 100 B x {sum(items)} / "
            f"{steps:,} = {alg_b:.3f} B), {(fetch_b + write_b) / (kt / kn) / 1e9:.0f} GB/s."]
    open(COUNTERS_MD, "w").write("\n".join(out) + "\n")
    json.dump({"kernel": pq, "workload": f"giants_100k, 100,000 particles x {steps} steps",
               "source_hash": src, "flops_per_particle_step": fpps,
               "bytes_per_particle_step": bpps, "fetch_factor": fetch_f, "write_factor": write_f,
               "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
               "active_particle_steps_per_launch": aps / launches, "summary": os.path.basename(COUNTERS_MD)},
              open(COUNTERS_JSON, "w"), indent=1)
    print("\n".join(out[-6:]))
    summarize_ephemeris(pmc_dir, tot, cnt, steps, src)


def summarize_resonant_counters(pmc_dir: str) -> None:
    """Write the resonant workload's counter summary (markdown) and its executed
    FP64 flops per active particle-step (json) from the rocprofv3 pass in
    pmc_dir/r1, made by `rocprofv3 --pmc <RES_PMC> --kernel-trace -f csv -d
    <pmc_dir>/r1 -o run -- python3 bench.py <RES_PMC_BENCH_ARGS>` with its
    output in <pmc_dir>/r1.log.  The resonant run's particle launches are the
    kernel variant with a one-step row prefetch (several wavefronts per SIMD);
    the small headline run before it uses the three-step one."""
    import collections
    import csv
    res_kernel = "particle_queue<4, 5, false, 1>"
    tot = collections.Counter()
    launches = 0
    for r in csv.DictReader(open(os.path.join(pmc_dir, "r1", "run_counter_collection.csv"))):
        if res_kernel in r["Kernel_Name"]:
            tot[r["Counter_Name"]] += float(r["Counter_Value"])
            if r["Counter_Name"] == "SQ_WAVES":
                launches += 1
    kt = 0.0
    for r in csv.DictReader(open(os.path.join(pmc_dir, "r1", "run_kernel_trace.csv"))):
        if res_kernel in r["Kernel_Name"]:
            kt += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    run = json.loads([x for x in open(os.path.join(pmc_dir, "r1.log")) if x.startswith("{")][-1])
    src = run["kernel_sources"]
    aps = run["resonant"]["active_particle_steps"]
    steps = int(RES_PMC_BENCH_ARGS.split()[-1])
    per = lambda c: 64 * tot[c] / aps
    fpps = per("SQ_INSTS_VALU_FLOPS_FP64")
    rate = fpps * aps / kt / 1e12
    out = [f"# particle_queue<4,5> counters -- resonant_200k, 200,000 particles x {steps:,} steps "
           f"({launches} launches)", "",
           "Command (`cd /tmp && export TMPDIR=/tmp` first), then `python3 bench.py "
           "--summarize-resonant-counters <out>` for this summary:", "",
           f"    timeout -s KILL 120 rocprofv3 --pmc {RES_PMC} --kernel-trace -f csv -d <out>/r1 "
           f"-o run -- python3 <repo>/bench.py {RES_PMC_BENCH_ARGS} > <out>/r1.log", "",
           f"Kernel sources of the counted run: `bench.kernel_source_hash()` = `{src}`.", "",
           f"Sums over the resonant run's {launches} particle launches ({res_kernel}; the "
           "1,024-particle headline run before it uses another variant and is left out), from "
           "`run_counter_collection.csv`:", "", "| counter | value |", "|---|---|"]
    for c, v in tot.items():
        out.append(f"| {c} | {v:.6g} |")
    out += ["", f"Derived ({aps:,} active particle-steps; kernel-trace time {kt * 1e3:.1f} ms):", "",
            f"* Executed FP64 per active particle-step (64 x instructions / particle-steps): "
            f"{per('SQ_INSTS_VALU_FMA_F64'):.1f} FMA, {per('SQ_INSTS_VALU_MUL_F64'):.1f} mul, "
            f"{per('SQ_INSTS_VALU_ADD_F64'):.1f} add, {per('SQ_INSTS_VALU_TRANS_F64'):.1f} "
            f"transcendental; flops (FMA = 2) {fpps:.1f}.",
            f"* FP64 rate under the profiler: {fpps:.1f} x {aps:.4g} / {kt * 1e3:.1f} ms = "
            f"{rate:.1f} TFLOP/s = {rate / FP64_PEAK_TFLOPS * 100:.0f}% of {FP64_PEAK_TFLOPS}."]
    open(RES_COUNTERS_MD, "w").write("\n".join(out) + "\n")
    json.dump({"kernel": "particle_queue<4,5>", "workload": f"resonant_200k, {steps} steps",
               "source_hash": src, "flops_per_particle_step": fpps,
               "summary": os.path.basename(RES_COUNTERS_MD)}, open(RES_COUNTERS_JSON, "w"), indent=1)
    print("\n".join(out[-3:]))


def summarize_ephemeris(pmc_dir: str, tot, cnt, steps: int, src: str) -> None:
    """The planet map's part of the same counter passes (one wavefront, serial
    in time), per step, and its kernel-trace time beside the particle kernel
    (pass 2) and alone (`python3 bench.py --ephemeris-only --nsteps 100000`
    under `rocprofv3 --kernel-trace -f csv -d <pmc_dir>/alone -o run`)."""
    import csv
    eph = "ephemeris_chunk<4>"
    g = lambda p, c: tot[(p, eph, c)]

    def trace(path):
        t, k, n = 0.0, 0, 0
        for r in csv.DictReader(open(path)):
            if "ephemeris_chunk" in r["Kernel_Name"]:
                t += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
                k += 1
        return t, k

    beside, nb = trace(os.path.join(pmc_dir, "p2", "run_kernel_trace.csv"))
    alone_csv = os.path.join(pmc_dir, "alone", "run_kernel_trace.csv")
    alone_steps = 100_000
    alone, na = trace(alone_csv) if os.path.exists(alone_csv) else (None, 0)
    per = lambda p, c: g(p, c) / steps
    flops = 64 * per("p1", "SQ_INSTS_VALU_FLOPS_FP64")
    out = [f"# ephemeris_chunk<4> counters -- the planet map of giants_100k (4 planets), {steps:,} steps "
           f"({cnt[('p1', eph, 'SQ_WAVES')]} launches, one wavefront each)", "",
           "From the same four counter passes as `particle_queue_giants_100k_counters.md` (commands "
           "there), which run the planet map beside the particle kernel; its time alone from "
           "`cd /tmp && export TMPDIR=/tmp; rocprofv3 --kernel-trace -f csv -d <out>/alone -o run -- "
           f"python3 <repo>/bench.py --ephemeris-only --nsteps {alone_steps}`; then "
           "`python3 bench.py --summarize-counters <out>`.", "",
           f"Kernel sources of the counted runs: `bench.kernel_source_hash()` = `{src}`.", "",
           "| counter | sum | per step |", "|---|---|---|"]
    for (p, lab, c), v in sorted(tot.items()):
        if lab == eph:
            out.append(f"| {c} | {v:.6g} | {v / steps:.1f} |")
    out += ["", "Derived, per step of the map (one wavefront; SQ cycle counters in units of 4 cycles):", "",
            f"* VALU instructions {per('p1', 'SQ_INSTS_VALU'):.0f}, of them FP64 FMA "
            f"{per('p1', 'SQ_INSTS_VALU_FMA_F64'):.0f}, mul {per('p1', 'SQ_INSTS_VALU_MUL_F64'):.0f}, "
            f"add {per('p1', 'SQ_INSTS_VALU_ADD_F64'):.0f}, transcendental "
            f"{per('p1', 'SQ_INSTS_VALU_TRANS_F64'):.0f}; SALU {per('p2', 'SQ_INSTS_SALU'):.0f}, SMEM "
            f"{per('p2', 'SQ_INSTS_SMEM'):.0f}; executed FP64 flops (all 64 lanes) {flops:.0f}.",
            f"* Wave cycles {4 * per('p2', 'SQ_WAVE_CYCLES'):.0f}: VALU issuing "
            f"{4 * per('p2', 'SQ_ACTIVE_INST_VALU'):.0f}, any instruction issuing "
            f"{4 * per('p2', 'SQ_ACTIVE_INST_ANY'):.0f}, waiting on a dependency or memory "
            f"{4 * per('p2', 'SQ_WAIT_ANY'):.0f}, waiting to issue "
            f"{4 * per('p2', 'SQ_WAIT_INST_ANY'):.0f}.",
            f"* Kernel-trace time beside the particle kernel (pass 2): {beside * 1e3:.2f} ms for "
            f"{steps:,} steps in {nb} launches = {beside / steps * 1e6:.3f} us per step."]
    if alone is not None:
        out.append(f"* Alone (no particle kernel): {alone * 1e3:.2f} ms for {alone_steps:,} steps in "
                   f"{na} launches = {alone / alone_steps * 1e6:.3f} us per step.")
    path = os.path.join(ROOT, "profiles", "ephemeris_chunk_giants_100k_counters.md")
    open(path, "w").write("\n".join(out) + "\n")
    print("\n".join(out[-4:]))


# rocprofv3 kernel-trace runs summarized by --summarize-traces DIR: subdirectory
# of DIR -> (summary under profiles/, title, bench.py arguments of the run)
TRACE_RUNS = {
    "tl": ("pipeline_giants_100k_1e6_timeline.md",
           "Pipeline timeline -- giants_100k, 100,000 particles x 1,000,000 steps (one benchmark run)",
           "--steps 1 --warmup 0 --no-cpu --no-adjoint --no-batched --no-resonant --no-handoff"),
    "k100k": ("particle_queue_giants_100k_kernel_trace.md",
              "particle_queue / ephemeris_chunk -- giants_100k, 100,000 particles x 100,000 steps",
              "--nsteps 100000 --steps 1 --warmup 0 --no-cpu --no-adjoint --no-batched --no-resonant "
              "--no-handoff"),
    "ad": ("ad_kernels_adjoint_16k_kernel_trace.md",
           "ad_segment / ad_reverse -- adjoint_16k, 16,384 particles x 100,000 steps, checkpoint 1,000",
           "--nsteps 1000 --n 1024 --steps 1 --warmup 0 --no-cpu --no-batched --no-resonant "
           "--no-handoff"),
    "batched": ("particle_batch_queue_batched_512_kernel_trace.md",
                "particle_batch_queue / ephemeris_batch -- 512 systems, 811,726 particles x 100,000 "
                "steps (one graph launch)",
                "--nsteps 1000 --n 1024 --steps 1 --warmup 0 --no-cpu --no-adjoint --no-resonant "
                "--no-handoff"),
    "res": ("particle_queue_resonant_200k_kernel_trace.md",
            "particle_queue / ephemeris_chunk -- resonant_200k, 200,000 particles x 1,000,000 steps",
            "--nsteps 1000 --n 1024 --steps 1 --warmup 0 --no-cpu --no-adjoint --no-batched "
            "--no-handoff"),
    "ho": ("encounter_run_giants_100k_handoff_kernel_trace.md",
           "particle_queue / encounter_run -- giants_100k with the close-encounter hand-off, "
           "100,000 particles x 1,000,000 steps, 16 substeps",
           "--nsteps 1000 --n 1024 --steps 1 --warmup 0 --no-cpu --no-adjoint --no-batched "
           "--no-resonant"),
}


def _trace_rows(path: str):
    import csv
    rows = []
    for r in csv.DictReader(open(path)):
        rows.append((r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    rows.sort(key=lambda x: x[1])
    return rows


def _short(name: str) -> str:
    """Kernel name without its argument list."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    i = name.find("(")
    return name[:i] if i > 0 else name


def summarize_traces(tdir: str) -> None:
    """Write the kernel-trace summaries of TRACE_RUNS from rocprofv3 runs made
    by `rocprofv3 --kernel-trace -f csv -d <tdir>/<key> -o run -- python3
    bench.py <args>` with stdout in <tdir>/<key>.log (no GPU use)."""
    import collections
    for key, (fname, title, args) in TRACE_RUNS.items():
        path = os.path.join(tdir, key, "run_kernel_trace.csv")
        if not os.path.exists(path):
            print(f"skipping {key}: no {path}")
            continue
        rows = _trace_rows(path)
        log = [x for x in open(os.path.join(tdir, key + ".log")) if x.startswith("{")]
        line = json.loads(log[-1]) if log else {}
        stats = collections.OrderedDict()
        for k, t0, t1 in rows:
            st = stats.setdefault(_short(k), [0, 0.0, 1e30, 0.0])
            d = (t1 - t0) * 1e-3
            st[0] += 1
            st[1] += d
            st[2] = min(st[2], d)
            st[3] = max(st[3], d)
        total = sum(v[1] for v in stats.values())
        out = [f"# {title}", "",
               "Command (from the repository root on the GPU box, `cd /tmp && export TMPDIR=/tmp` "
               "first), then `python3 bench.py --summarize-traces <out>` for this summary:", "",
               f"    rocprofv3 --kernel-trace -f csv -d <out>/{key} -o run -- python3 <repo>/bench.py "
               f"{args} > <out>/{key}.log", "",
               f"Kernel sources: `bench.kernel_source_hash()` = `{line.get('kernel_sources', '?')}`.", "",
               "All dispatches of the process, from `run_kernel_trace.csv`:", "",
               "| kernel | calls | total ms | average us | min us | max us | % of kernel time |",
               "|---|---|---|---|---|---|---|"]
        for k, (c, tot, mn, mx) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
            out.append(f"| {k} | {c} | {tot / 1e3:.2f} | {tot / c:.1f} | {mn:.1f} | {mx:.1f} | "
                       f"{100 * tot / total:.2f} |")
        out += [""] + _trace_details(key, rows, line)
        open(os.path.join(ROOT, "profiles", fname), "w").write("\n".join(out) + "\n")
        print(f"wrote profiles/{fname}")


def _trace_details(key, rows, line):
    """Figures of one trace beyond the per-kernel table."""
    pq = [(t0, t1) for k, t0, t1 in rows if "particle_queue" in k]
    eph = [(t0, t1) for k, t0, t1 in rows if "ephemeris_chunk" in k]
    out = []
    if key in ("tl", "k100k", "res") and pq:
        kern = line.get("kernel", {})
        if key == "res":
            r = line.get("resonant", {})
            out += [f"Resonant line of the same run: {r.get('value', 0):.4g} active particle-steps/s end "
                    f"to end, {r.get('particle_steps_per_s_kernels_only', 0):.4g} kernels only, "
                    f"{r.get('run_ms', 0):.1f} ms, survivors {r.get('survivors')}.", ""]
            return out
        avg = sum(t1 - t0 for t0, t1 in pq) / len(pq) * 1e-6
        out += [f"Bench line of the same run: {line.get('value', 0):.4g} active particle-steps/s, "
                f"{line.get('ms_per_step', 0):.1f} ms per run; particle kernel "
                f"{kern.get('launches')} launches, HIP-event average {kern.get('avg_launch_ms', 0):.3f} ms "
                f"per launch against rocprofv3's {avg:.3f} ms.", ""]
        if key == "tl":
            span = (max(t1 for _, t1 in pq + eph) - min(t0 for t0, _ in pq + eph)) * 1e-6
            bp = sum(t1 - t0 for t0, t1 in pq) * 1e-6
            be = sum(t1 - t0 for t0, t1 in eph) * 1e-6
            gaps = sum(max(0, pq[i + 1][0] - pq[i][1]) for i in range(len(pq) - 1)) * 1e-6
            out += [f"Span of the run {span:.1f} ms; particle kernels busy {bp:.1f} ms "
                    f"({100 * bp / span:.0f}%), planet map busy {be:.1f} ms ({100 * be / span:.0f}%); "
                    f"gaps between particle launches {gaps:.1f} ms in total.", "",
                    "Average duration per tenth of the run (launch 0 covers 1,024 steps, the others "
                    "8,192 but the last):", "",
                    "| launches | particle_queue us | ephemeris_chunk us |", "|---|---|---|"]
            m = min(len(pq), len(eph))
            step = max(1, m // 10)
            for a in range(0, m, step):
                b = min(m, a + step)
                out.append(f"| {a}-{b - 1} | {sum(t1 - t0 for t0, t1 in pq[a:b]) / (b - a) / 1e3:.0f} | "
                           f"{sum(t1 - t0 for t0, t1 in eph[a:b]) / (b - a) / 1e3:.0f} |")
            out.append("")
    if key == "ad":
        a = line.get("adjoint", {})
        seg = [(t0, t1) for k, t0, t1 in rows if "ad_segment" in k]
        rev = [(t0, t1) for k, t0, t1 in rows if "ad_reverse" in k]
        out += [f"Adjoint line of the same run: forward {a.get('forward_s', 0) * 1e3:.1f} ms, backward "
                f"{a.get('backward_s', 0) * 1e3:.1f} ms (x{a.get('backward_over_forward', 0):.2f}); "
                f"production forward {a.get('production_forward_s', 0) * 1e3:.1f} ms "
                f"(backward over it x{a.get('backward_over_production_forward', 0):.2f}).", ""]
        if rev:
            # the timed backward pass: its sweeps and recomputations are the
            # last nseg of each (a warm-up pass and the forward's segments
            # come before them)
            import re
            m = re.search(r"(\d+) steps, checkpoint every (\d+)", a.get("workload", ""))
            nseg = -(-int(m.group(1)) // int(m.group(2))) if m else len(rev)
            rev, rec = rev[-nseg:], seg[-nseg:]
            ov = sum(max(0, min(t1, u1) - max(t0, u0)) for t0, t1 in rec for u0, u1 in rev)
            span = (max(t1 for _, t1 in rev + rec) - min(t0 for t0, _ in rev + rec)) * 1e-6
            out += [f"Timed backward pass ({nseg} segments): sweeps (ad_reverse, caller's stream) "
                    f"{sum(t1 - t0 for t0, t1 in rev) * 1e-6:.1f} ms busy, {sum(t1 - t0 for t0, t1 in rev) * 1e-3 / nseg:.0f} us "
                    f"each; recomputations (ad_segment, library stream) "
                    f"{sum(t1 - t0 for t0, t1 in rec) * 1e-6:.1f} ms busy, {ov * 1e-6:.1f} ms of it beside a "
                    f"sweep; span {span:.1f} ms.", ""]
    if key == "ho":
        h = line.get("handoff", {})
        enc = [(t0, t1) for k, t0, t1 in rows if "encounter_run" in k]
        ov = 0
        for t0, t1 in enc:          # overlap of each encounter launch with the particle launches
            ov += sum(max(0, min(t1, u1) - max(t0, u0)) for u0, u1 in pq)
        out += [f"Hand-off line of the same run: {h.get('value', 0):.4g} active particle-steps/s, "
                f"{h.get('run_ms', 0):.1f} ms, {h.get('handoffs')} hand-offs, removed by reason "
                f"{h.get('removed_by_reason')}, survivors {h.get('survivors')}.", ""]
        if enc:
            out += [f"encounter_run: {len(enc)} launches, {sum(t1 - t0 for t0, t1 in enc) * 1e-6:.1f} ms "
                    f"busy, {ov * 1e-6:.1f} ms of it beside a particle_queue launch; particle_queue "
                    f"{sum(t1 - t0 for t0, t1 in pq) * 1e-6:.1f} ms busy.", "",
                    "encounter_run durations in launch order, ms:", "",
                    "    " + " ".join(f"{(t1 - t0) * 1e-6:.0f}" for t0, t1 in enc), ""]
    if key == "batched":
        b = line.get("batched", {})
        out += [f"Many-system line of the same run: {b.get('value', 0):.4g} active particle-steps/s, "
                f"graph {b.get('graph_ms', 0):.1f} ms by HIP events, tuned {b.get('tuned')}, "
                f"call {b.get('call_s_incl_setup_and_tuning', 0):.2f} s including set-up and tuning.", ""]
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, steps_sample: int, n_single: int):
    """The oracle on the host: every particle of the workload for steps_sample
    steps on all threads, then n_single particles for the same steps on one
    thread."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    eph = oracle.ephemeris(w.mu0, w.mu, w.rp, w.vp, steps_sample, w.dt)
    t1 = time.perf_counter()

    def rate(sub, nthreads):
        res = oracle.particles(sub.mu0, sub.mu, sub.rcrit, sub.rmax, eph.table, sub.dt, sub.r,
                               sub.v, steps_sample, kepler_iters=sub.kepler_iters,
                               nthreads=nthreads)
        d = res.deact_step
        active = int(np.where(d < 0, steps_sample, d).sum())
        return active, res.seconds

    cores = oracle.max_threads()
    a_all, s_all = rate(w, cores)
    a_one, s_one = rate(w.subset(n=n_single), 1)
    oracle.max_threads(cores)
    return {"value": a_all / s_all, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"all {w.n} particles x {steps_sample} steps of the same workload on {cores} "
                      f"threads ({a_all} active particle-steps, {s_all:.1f} s; planet map "
                      f"{t1 - t0:.2f} s, serial, not counted)",
            "single_core": {"value": a_one / s_one, "unit": "particle-steps/s",
                            "sample": f"first {n_single} particles x {steps_sample} steps, 1 thread "
                                      f"({s_one:.1f} s)"},
            "cpu_model": cpu_model(),
            "paper_speedup": PAPER_SPEEDUP}


def adjoint_ratio(P, W, torch, nsteps: int, n: int, ckpt: int):
    """Forward (with checkpoints) and backward of loss = sum |r_T|^2 on the
    16,384-particle four-planet workload; returns times and their ratio, also
    against the production forward (tpm_integrate, no checkpoints) of the same
    run."""
    from paper_2011_03484_amd import autograd as AG
    w = W.adjoint_16k(n=n)
    # the production forward: the same particles and steps through tpm_integrate
    p = P.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters)
    p.set_central(w.mu0)
    p.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    p.set_particles(w.r, w.v)
    p.integrate(2 * ckpt, w.dt)
    p.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    p.set_particles(w.r, w.v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.integrate(nsteps, w.dt)
    torch.cuda.synchronize()
    prod_s = time.perf_counter() - t0
    p.close()
    s = P.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters)
    s.set_central(w.mu0)
    s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    r0 = torch.tensor(w.r, dtype=torch.float64, device="cuda").requires_grad_(True)
    v0 = torch.tensor(w.v, dtype=torch.float64, device="cuda").requires_grad_(True)
    # warm-up on a short run
    rT, vT, _, _ = AG.integrate(s, r0, v0, 2 * ckpt, w.dt, ckpt)
    (rT ** 2).sum().backward()
    r0.grad = v0.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rT, vT, step, reason = AG.integrate(s, r0, v0, nsteps, w.dt, ckpt)
    loss = (rT ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    survivors = int((reason == 0).sum().item())
    s.close()
    return {"workload": f"adjoint_16k: {n} particles, 4 planets, {nsteps} steps, checkpoint every "
                        f"{ckpt}, loss = sum |r_T|^2",
            "forward_s": t1 - t0, "backward_s": t2 - t1, "backward_over_forward": (t2 - t1) / (t1 - t0),
            "production_forward_s": prod_s,
            "backward_over_production_forward": (t2 - t1) / prod_s,
            "survivors": survivors}


def batched_run(P, W, nsteps: int):
    """512 independent systems (Np 1..8, ~0.86M particles) in one graph launch."""
    systems = W.make_batched(nsteps=nsteps)
    t0 = time.perf_counter()
    res, st = P.batch_integrate(systems, nsteps=nsteps, strict=False)
    t1 = time.perf_counter()
    n = sum(w.n for w in systems)
    return {"workload": f"batched_512: 512 systems, Np U{{1..8}}, {n} particles, dt = P_inner/30, "
                        f"{nsteps} steps, one HIP-graph launch",
            "value": st["active_particle_steps"] / (st["particle_ms"] / 1e3),
            "unit": "particle-steps/s", "graph_ms": st["particle_ms"],
            "call_s_incl_setup_and_tuning": t1 - t0,
            "active_particle_steps": st["active_particle_steps"],
            "systems_with_planet_close_approach": int((st["planet_flag"] != -1).sum()),
            "tuned": {"block_threads": st["block_threads"], "chunk_steps": st["chunk_steps"],
                      "sub_chunks": st["sub_chunks"], "waves_per_simd": st["waves_per_simd"],
                      "resync_chunks": st["resync_chunks"]}}


def resonant_run(P, W, torch, nsteps: int):
    """The 200,000-particle resonant workload (a 54-64 au, e 0.1-0.5, i up to
    20 degrees; removal within one Hill radius or beyond 1000 au) for nsteps
    steps: a decaying population with compaction, end to end."""
    w = W.resonant_200k()
    s = P.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters, time_kernels=True)
    s.set_central(w.mu0)
    s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    s.set_particles(w.r, w.v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.integrate(nsteps, w.dt)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = s.stats()
    s.close()
    kernel_rate = st["active_particle_steps"] / (st["particle_kernel_ms"] / 1e3)
    cf = counter_figures(RES_COUNTERS_JSON)
    executed = None
    if cf:
        tf = cf["flops_per_particle_step"] * kernel_rate / 1e12
        executed = {"flops_per_particle_step": cf["flops_per_particle_step"], "tflops": tf,
                    "frac": tf / FP64_PEAK_TFLOPS,
                    "source": "SQ_INSTS_VALU_FLOPS_FP64 of the committed counter run of this "
                              "workload on the same kernel sources, per active particle-step, over "
                              "this run's particle-kernel time"}
    return {"workload": f"resonant_200k: 200,000 particles, 4 planets, dt = 120 d, {nsteps} steps "
                        f"(the first {nsteps / 1e7:.0%} of its 1e7-step length)",
            "value": st["active_particle_steps"] / secs, "unit": "particle-steps/s",
            "run_ms": secs * 1e3,
            "particle_steps_per_s_kernels_only": kernel_rate,
            "active_particle_steps": st["active_particle_steps"],
            "removed_by_reason": st["count_by_reason"][1:], "survivors": st["count_by_reason"][0],
            "compactions": st["compactions"], "executed_fp64": executed}


def handoff_run(P, W, torch, nsteps: int, substeps: int = 16, r_rem: float = 0.05):
    """The headline workload with the close-encounter hand-off: a particle
    within 0.5 au of a planet moves to the encounter integrator (substeps
    substeps per step, planets on their Hermite interpolants) and is removed
    within r_rem; the encounter stream runs behind the main one."""
    w = W.giants_100k()
    s = P.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters, time_kernels=True,
                     handoff_substeps=substeps, universal_drift=True)
    s.set_central(w.mu0)
    s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
    s.set_removal_radii([r_rem] * w.np_)
    s.set_particles(w.r, w.v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.integrate(nsteps, w.dt)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = s.stats()
    s.close()
    return {"workload": f"giants_100k with the close-encounter hand-off: 100,000 particles, "
                        f"4 planets, dt = 120 d, {nsteps} steps, hand-off within 0.5 au, "
                        f"{substeps} substeps per encounter step, removal within {r_rem} au",
            "value": st["active_particle_steps"] / secs, "unit": "particle-steps/s",
            "run_ms": secs * 1e3, "handoffs": st["handoffs"],
            "particle_kernel_ms": st["particle_kernel_ms"],
            "active_particle_steps": st["active_particle_steps"],
            "removed_by_reason": st["count_by_reason"][1:], "survivors": st["count_by_reason"][0]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nsteps", type=int, default=1_000_000, help="time steps per run")
    ap.add_argument("--n", type=int, default=100_000, help="particles")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--resync", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--sub-chunks", type=int, default=0, help="work items per tile per chunk (0 = library default)")
    ap.add_argument("--waves-per-simd", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=10000,
                    help="steps of the oracle's all-particle CPU sample")
    ap.add_argument("--cpu-single", type=int, default=2048,
                    help="particles of the oracle's one-thread CPU sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=100_000)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=100_000)
    ap.add_argument("--no-resonant", action="store_true")
    ap.add_argument("--resonant-steps", type=int, default=1_000_000)
    ap.add_argument("--no-handoff", action="store_true")
    ap.add_argument("--handoff-steps", type=int, default=1_000_000)
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device with a plain copy "
                         "kernel (the reference for scaling HBM byte counters)")
    ap.add_argument("--ephemeris-only", action="store_true",
                    help="run only the planet map of the workload for --nsteps steps (its time "
                         "alone) and print one JSON line")
    ap.add_argument("--summarize-traces", metavar="DIR",
                    help="write the kernel-trace summaries under profiles/ from rocprofv3 "
                         "--kernel-trace runs in DIR (see TRACE_RUNS), then exit (no GPU use)")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="write the counter summary under profiles/ from rocprofv3 --pmc passes "
                         "p1..p4 in DIR, then exit (no GPU use)")
    ap.add_argument("--summarize-resonant-counters", metavar="DIR",
                    help="write the resonant workload's counter summary under profiles/ from the "
                         "rocprofv3 --pmc pass r1 in DIR, then exit (no GPU use)")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.summarize_resonant_counters:
        summarize_resonant_counters(args.summarize_resonant_counters)
        return
    if args.summarize_traces:
        summarize_traces(args.summarize_traces)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X "
              "(multi-GPU sharding is described in the design notes, not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2011_03484_amd as P
    from paper_2011_03484_amd import workloads as W

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.init()
    w = W.giants_100k(n=args.n)
    T = args.nsteps
    if args.ephemeris_only:
        s = P.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters, chunk_steps=args.chunk)
        s.set_central(w.mu0)
        s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
        s.planet_table(1024, w.dt)
        t0 = time.perf_counter()
        s.planet_table(T, w.dt)
        t1 = time.perf_counter()
        print(json.dumps({"mode": "ephemeris-only", "workload": "giants_100k planets", "steps": T,
                          "call_s_incl_table_copy": t1 - t0}))
        return
    sims = []
    for _ in range(args.warmup + args.steps):
        s = P.Simulation(r_escape=w.rmax, kepler_iters=w.kepler_iters, chunk_steps=args.chunk,
                         resync_chunks=args.resync, block_threads=args.block, time_kernels=True,
                         sub_chunks=args.sub_chunks, waves_per_simd=args.waves_per_simd)
        s.set_central(w.mu0)
        s.set_planets(w.mu, w.rp, w.vp, w.rcrit)
        s.set_particles(w.r, w.v)
        sims.append(s)
    for i in range(args.warmup):
        sims[i].integrate(T, w.dt)
        print(f"warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        sims[i].integrate(T, w.dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = [sims[i].stats() for i in range(args.warmup, args.warmup + args.steps)]
    secs = t1 - t0
    aps = sum(s["active_particle_steps"] for s in stats)
    kern_ms = sum(s["particle_kernel_ms"] for s in stats)
    launches = sum(s["chunks"] for s in stats)
    eph_ms = sum(s["ephemeris_ms"] for s in stats)
    pstream_ms = sum(s["particle_ms"] for s in stats)
    cf = counter_figures()
    fpps = ALGORITHMIC_FLOPS_PER_PARTICLE_STEP.get(w.np_)
    achieved = fpps * aps / (kern_ms / 1e3) / 1e12 if fpps and kern_ms > 0 else None
    traffic = cf["bytes_per_particle_step"] * aps / max(launches, 1) if cf is not None else None
    executed = None
    if cf is not None and kern_ms > 0:
        ex = cf["flops_per_particle_step"] * aps / (kern_ms / 1e3) / 1e12
        executed = {"flops_per_particle_step": cf["flops_per_particle_step"], "tflops": ex,
                    "frac": ex / FP64_PEAK_TFLOPS,
                    "source": "SQ_INSTS_VALU_FLOPS_FP64 of the committed counter runs on the same "
                              "kernel sources, per active particle-step, over this run's kernel time"}
    line = {
        "metric": "FP64 particle-steps/sec and % FP64 peak, 1 MI355X; adjoint/forward cost ratio",
        "value": aps / secs,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "giants_100k: Sun + 4 giant planets, 100,000 particles a~U[20,29] au, "
                               "dt=120 d, 1e6 steps per run" if (T == 1_000_000 and args.n == 100_000)
                   else f"giants_100k reduced: {args.n} particles, {T} steps per run",
                   "particles": args.n, "planets": w.np_, "time_steps": T, "dt_days": 120.0,
                   "kepler_iters": w.kepler_iters},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS if achieved else None,
                     "traffic": traffic},
        "kernel": {"name": "particle_queue<4,5>", "launches": launches,
                   "avg_launch_ms": kern_ms / max(launches, 1),
                   "algorithmic_flops_per_particle_step": fpps,
                   "executed_fp64": executed,
                   "particle_steps_per_s_kernels_only": aps / (kern_ms / 1e3) if kern_ms else None,
                   "particle_stream_ms": pstream_ms, "ephemeris_stream_ms": eph_ms},
        # % of the FP64 vector peak as the counters measure it (executed FP64
        # flops over kernel time); null when the counters predate the sources
        "fp64_peak_frac_executed": executed["frac"] if executed else None,
        "active_particle_steps": aps,
        "survivors_per_run": [s["count_by_reason"][0] for s in stats],
        "run_ms": [round(s["wall_ms"], 1) for s in stats],
        "kernel_sources": kernel_source_hash(),
    }
    for s in sims:
        s.close()
    if args.copy_calibration_mb > 0:
        # a plain device copy of known size, its source evicted from the
        # last-level cache first by writing a larger buffer
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        flush = torch.empty(4 * nbytes // 8, dtype=torch.float64, device="cuda")
        flush.fill_(2.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del flush
        line["copy_calibration_bytes"] = nbytes
    if not args.no_adjoint:
        line["adjoint"] = adjoint_ratio(P, W, torch, args.adjoint_steps, 16_384, 1000)
        print("adjoint done", file=sys.stderr, flush=True)
    if not args.no_batched:
        line["batched"] = batched_run(P, W, args.batched_steps)
        print("batched done", file=sys.stderr, flush=True)
    if not args.no_resonant:
        line["resonant"] = resonant_run(P, W, torch, args.resonant_steps)
        print("resonant done", file=sys.stderr, flush=True)
    if not args.no_handoff:
        line["handoff"] = handoff_run(P, W, torch, args.handoff_steps)
        print("handoff done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, args.cpu_single)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
