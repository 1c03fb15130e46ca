#!/usr/bin/env python3
"""Throughput of the MI355X PairHMM forward path on the genome-scale
synthetic WGS-like workload (the fourth synthetic configuration: 150 bp
reads, 2-16 variant haplotypes of 150-600 bp per region, lognormal read
counts with mean 40, Phred 2-41 base qualities, FP32 with FP64 reruns).

One step = one pass of the whole hot path over the batch, which is resident
in HBM before timing starts: device-side grouping/packing of pairs, the
FP32 short-pair kernels, the FP64 reruns and the long-pair kernel.

Prints one JSON line (see the design notes for every field).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import math
import multiprocessing as mp
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "GCUPS (PairHMM cells/s) vs FP32 VALU roofline; p50/p99 region latency"
FLOPS_PER_CELL = 12          # eq.2 as written, an FMA counted as two flops
FP32_PEAK_TFLOPS = 157.3     # MI355X vector FP32 (vendor figure)

_BATCH = None  # inherited by the oracle worker processes

# HBM traffic of the FP32 short-kernel family, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs of this script (see summarize_traffic); valid only for the
# kernel sources and workload it was taken on.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_short_fp32_wgs.md")
COUNTERS_PROFILE = os.path.join(ROOT, "profiles", "valu_counters_short_fp32_wgs.md")
TRACE_PROFILE = os.path.join(ROOT, "profiles", "short_kernels_wgs_1M_regions.md")
CSRC = os.path.join(ROOT, "paper_2606_25738_amd", "csrc")
N_CLASSES = 21               # column classes of the short kernels (N = 4, 5, ..., 24)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _oracle_chunk(idx):
    import oracle
    t = time.process_time()
    v = oracle.forward_pairs(_BATCH, idx, rescale=True)
    return v, time.process_time() - t


def _cpu_model():
    """The host CPU's model name as lscpu and /proc/cpuinfo report it (either
    may be shortened inside a container), or None."""
    names = []
    try:
        import subprocess
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        for line in r.stdout.splitlines():
            if line.strip().startswith("Model name"):
                names.append(line.split(":", 1)[1].strip())
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    names.append(line.split(":", 1)[1].strip())
                    break
    except OSError:
        pass
    names = list(dict.fromkeys(n for n in names if n))
    return max(names, key=len) if names else None


def _host_cpus():
    """Logical CPUs of the host and those this process may run on."""
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = None
    return os.cpu_count(), aff


def sample_regions(batch, n_regions, seed=123):
    nreg = len(batch["region_pairs"]) - 1
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(nreg, size=min(n_regions, nreg), replace=False))


def sample_pairs(batch, n_regions, seed=123):
    rp = batch["region_pairs"]
    regs = sample_regions(batch, n_regions, seed)
    return np.concatenate([np.arange(rp[r], rp[r + 1]) for r in regs]).astype(np.int64), len(regs)


def genotype_parity(batch, n_regions, ovals, gl, n_check=300):
    """Genotype likelihoods of the first n_check regions of the oracle's
    sample: the oracle's genotyping of the oracle's forward values against
    the GPU's genotyping of the GPU's forward output (gl, host copy).  Each
    read's term moves by at most its likelihoods' error, so the tolerance is
    1e-4 per read (the FP32 bound) plus 1e-12 relative."""
    import oracle
    import paper_2606_25738_amd as phmm
    rr, rh = batch["region_reads"], batch["region_haps"]
    H_all = np.diff(rh).astype(np.int64)
    go, _ = phmm.genotype_offsets(H_all)
    regs = sample_regions(batch, n_regions)
    off, worst, ok = 0, 0.0, True
    for k, g in enumerate(regs):
        R, H = int(rr[g + 1] - rr[g]), int(H_all[g])
        if k < n_check:
            ref = oracle.genotype_region(ovals[off:off + R * H].reshape(R, H))
            got = gl[int(go[g]):int(go[g]) + len(ref)]
            err = np.abs(got - ref)
            worst = max(worst, float((err / max(R, 1)).max()))
            ok &= bool(np.all(err <= 1e-4 * R + 1e-12 * np.abs(ref)))
        off += R * H
    return dict(regions=min(n_check, len(regs)), max_err_per_read=worst, ok=ok)


def run_oracle(batch, idx, cores):
    global _BATCH
    _BATCH = batch
    chunks = np.array_split(idx, max(1, cores * 8))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_chunk, chunks)
    wall = time.perf_counter() - t0
    vals = np.concatenate([r[0] for r in res])
    cpu = sum(r[1] for r in res)
    return vals, wall, cpu


# sources that decide what the FP32 short kernels and the packer do
TRAFFIC_SOURCES = ("phmm_short.hip", "phmm_dev.h", "phmm_internal.h", "phmm_pack.hip")


def sources_digest():
    """sha256 over the kernel sources (any change invalidates stored counters)."""
    h = hashlib.sha256()
    for f in sorted(os.path.join(CSRC, n) for n in TRAFFIC_SOURCES):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _pmc_rows(path, counter):
    with open(path, newline="") as fh:
        return [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]


def _step_dispatches(path):
    """Counter values (summed over a dispatch's rows) of the FP32 short-kernel
    launches of the last forward pass in a rocprofv3 counter CSV: the last 42
    dispatches of `short_kernel<float, c, kind>` by dispatch id.  Earlier
    dispatches (the pack-cost autotuning on a sample) are left out."""
    by = {}
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            m = re.search(r"short_kernel<float, (\d+), (\d+)>", r["Kernel_Name"])
            if not m:
                continue
            d = by.setdefault(int(r["Dispatch_Id"]), dict(
                cls=int(m.group(1)), kind=int(m.group(2)),
                ns=int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    ids = sorted(by)[-2 * N_CLASSES:]
    if len(ids) != 2 * N_CLASSES:
        raise SystemExit("%s: %d FP32 short-kernel dispatches, expected at least %d"
                         % (path, len(ids), 2 * N_CLASSES))
    return [by[i] for i in ids]


def summarize_traffic(fetch_csv, write_csv, out_path, regions, calib_mib, commands):
    """Writes the traffic profile from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE) of `bench.py --steps 1 --warmup 0 --fp64-steps 0 --no-cpu`.

    Counter values are KiB per dispatch.  Each counter is scaled by the ratio
    of the known size of the calibration copy (calib_mib read, calib_mib
    written) to what the same counter reads for that copy kernel."""
    res = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _pmc_rows(path, name)
        calib = [float(r["Counter_Value"]) for r in rows if "copy_calib_kernel" in r["Kernel_Name"]]
        if not calib:
            raise SystemExit("no copy_calib_kernel dispatch in %s" % path)
        factor = calib_mib * 1024.0 / calib[-1]
        per = {}
        for d in _step_dispatches(path):
            per[d["cls"]] = per.get(d["cls"], 0.0) + d[name]
        res[name] = dict(factor=factor, calib_kib=calib[-1], per_class=per)
    f, w = res["FETCH_SIZE"], res["WRITE_SIZE"]
    fetch_b = sum(f["per_class"].values()) * 1024.0 * f["factor"]
    write_b = sum(w["per_class"].values()) * 1024.0 * w["factor"]
    lines = ["# HBM traffic of the FP32 short-pair kernels, genome-scale WGS-like batch", "",
             "Commands (repository root, one MI355X):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", "Workload: %d regions, one step (42 launches of `short_kernel<float, c, kind>`: the fast"
              " and the general FP32 kernel of each class; counts per class summed over both). Only the"
              " launches of the last forward pass count (the pack-cost autotuning before it runs the"
              " same kernels on a sample)." % regions,
              "Counters are KiB per dispatch. Scale factor = known bytes of the calibration copy",
              "(`copy_calib_kernel`, %d MiB read and %d MiB written) / the counter's reading for it." %
              (calib_mib, calib_mib), "",
              "| class c (N = 4 + c) | FETCH_SIZE KiB | WRITE_SIZE KiB |", "|---:|---:|---:|"]
    for c in sorted(set(f["per_class"]) | set(w["per_class"])):
        lines.append("| %d | %.1f | %.1f |" % (c, f["per_class"].get(c, 0.0), w["per_class"].get(c, 0.0)))
    lines += ["", "Calibration copy: FETCH_SIZE %.1f KiB, WRITE_SIZE %.1f KiB for %d KiB each way." %
              (f["calib_kib"], w["calib_kib"], calib_mib * 1024),
              "", "Values read by bench.py:", "",
              "- regions: %d" % regions,
              "- fetch_factor: %.6f" % f["factor"],
              "- write_factor: %.6f" % w["factor"],
              "- fetch_bytes_per_step: %.6e" % fetch_b,
              "- write_bytes_per_step: %.6e" % write_b,
              "- traffic_bytes_per_step: %.6e" % (fetch_b + write_b),
              "- sources_sha256: %s" % sources_digest(), ""]
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32",
                 "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_FLOPS_FP32",
                 "SQ_INSTS_SALU", "SQ_BUSY_CU_CYCLES", "GRBM_GUI_ACTIVE")


def summarize_counters(pmc_csv, bench_json, out_path, commands):
    """Writes the instruction-count profile of the FP32 short kernels from one
    rocprofv3 --pmc run with VALU_COUNTERS, using the cell count from the JSON
    line the profiled bench.py run printed.  SQ counters are summed over all
    shader engines; GRBM_GUI_ACTIVE over the 8 XCDs (so the clock is it / 8 /
    the dispatch's duration); SQ_BUSY_CU_CYCLES reads as CU-cycles summed over
    the CUs (it agrees with 256 CUs x that clock x the duration)."""
    rec = None
    with open(bench_json) as fh:
        for line in fh:
            if line.startswith("{"):
                rec = json.loads(line)
    if rec is None:
        raise SystemExit("no JSON line in %s" % bench_json)
    cells = int(rec["config"]["cells"])
    rows = _step_dispatches(pmc_csv)
    tot = {c: sum(d.get(c, 0.0) for d in rows) for c in VALU_COUNTERS}
    ns = sum(d["ns"] for d in rows)
    fast = [d for d in rows if d["kind"] == 0]
    lines = ["# VALU instruction counts of the FP32 short-pair kernels, genome-scale WGS-like batch", "",
             "Commands (repository root, one MI355X):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", "Workload: %d regions, %d pairs, %.6g cells; one forward pass (42 launches of"
              " `short_kernel<float, c, kind>`, kind 0 the fast and 1 the general FP32 kernel)."
              % (rec["config"]["regions"], rec["config"]["pairs"], cells),
              "SQ counters are wave-instructions summed over the shader engines; the clock is"
              " GRBM_GUI_ACTIVE / 8 XCDs / the dispatch's duration (under counter collection);"
              " VALU per CU-clock = SQ_INSTS_VALU / SQ_BUSY_CU_CYCLES.", "",
              "| class c (N = 4 + c) | ms | VALU | FMA_F32 | MUL_F32 | ADD_F32 | INT32 | SALU |"
              " VALU per CU-clock | clock GHz |",
              "|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for d in fast:
        lines.append("| %d | %.2f | %.4g | %.4g | %.4g | %.4g | %.4g | %.4g | %.3f | %.2f |" % (
            d["cls"], d["ns"] / 1e6, d["SQ_INSTS_VALU"], d["SQ_INSTS_VALU_FMA_F32"],
            d["SQ_INSTS_VALU_MUL_F32"], d["SQ_INSTS_VALU_ADD_F32"], d["SQ_INSTS_VALU_INT32"],
            d["SQ_INSTS_SALU"], d["SQ_INSTS_VALU"] / max(1.0, d["SQ_BUSY_CU_CYCLES"]),
            d["GRBM_GUI_ACTIVE"] / 8.0 / max(1, d["ns"])))
    lane = 64.0 * tot["SQ_INSTS_VALU"] / cells
    fp = 64.0 * (tot["SQ_INSTS_VALU_FMA_F32"] + tot["SQ_INSTS_VALU_MUL_F32"]
                 + tot["SQ_INSTS_VALU_ADD_F32"]) / cells
    lines += ["", "Per useful cell over the pass (padding lanes and per-row work included):", "",
              "- valu_lane_instructions_per_cell: %.3f" % lane,
              "- fp32_fma_mul_add_lane_instructions_per_cell: %.3f" % fp,
              "- int32_lane_instructions_per_cell: %.3f" % (64.0 * tot["SQ_INSTS_VALU_INT32"] / cells),
              "- fp32_flops_counter_per_cell: %.4f (the counter counts per wave-instruction; x 64 lanes: %.2f,"
              " against 2 x FMA + MUL + ADD from the instruction counters x 64: %.2f)"
              % (tot["SQ_INSTS_VALU_FLOPS_FP32"] / cells, 64.0 * tot["SQ_INSTS_VALU_FLOPS_FP32"] / cells,
                 64.0 * (2.0 * tot["SQ_INSTS_VALU_FMA_F32"] + tot["SQ_INSTS_VALU_MUL_F32"]
                         + tot["SQ_INSTS_VALU_ADD_F32"]) / cells),
              "- algorithmic_flops_per_cell: %d" % FLOPS_PER_CELL,
              "- valu_per_cu_clock: %.3f" % (tot["SQ_INSTS_VALU"] / max(1.0, tot["SQ_BUSY_CU_CYCLES"])),
              "- clock_ghz: %.3f" % (tot["GRBM_GUI_ACTIVE"] / 8.0 / max(1, ns)),
              "- pass_ms_under_counters: %.2f" % (ns / 1e6),
              "- sources_sha256: %s" % sources_digest(), ""]
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


LDS_COUNTERS = ("SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_INSTS_VALU",
                "SQ_BUSY_CU_CYCLES", "GRBM_GUI_ACTIVE")
LDS_PROFILE = os.path.join(ROOT, "profiles", "lds_counters_short_fp32_wgs.md")


def summarize_lds(pmc_csv, bench_json, out_path, commands):
    """Writes the LDS profile of the FP32 short kernels from one rocprofv3
    --pmc run with LDS_COUNTERS: LDS instructions per cell, bank-conflict
    cycles (SQ_LDS_BANK_CONFLICT, summed over the shader engines) per LDS
    instruction and as a share of the cycles the LDS was busy with indexed
    operations (SQ_LDS_IDX_ACTIVE), per class and over the pass."""
    rec = None
    with open(bench_json) as fh:
        for line in fh:
            if line.startswith("{"):
                rec = json.loads(line)
    if rec is None:
        raise SystemExit("no JSON line in %s" % bench_json)
    cells = int(rec["config"]["cells"])
    rows = _step_dispatches(pmc_csv)
    tot = {c: sum(d.get(c, 0.0) for d in rows) for c in LDS_COUNTERS}
    fast = [d for d in rows if d["kind"] == 0]
    lines = ["# LDS counters of the FP32 short-pair kernels, genome-scale WGS-like batch", "",
             "Commands (repository root, one MI355X):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", "Workload: %d regions, %d pairs, %.6g cells; one forward pass (42 launches of"
              " `short_kernel<float, c, kind>`; the table shows the fast kernel of each class, the"
              " totals include the general ones). SQ counters summed over the shader engines;"
              " LDS instructions are wave-instructions (x 64 for lane counts)."
              % (rec["config"]["regions"], rec["config"]["pairs"], cells), "",
              "| class c (N = 4 + c) | ms | LDS instructions | LDS per 100 VALU | bank-conflict cycles |"
              " conflict cycles per LDS instruction | conflict share of LDS-busy cycles |",
              "|---:|---:|---:|---:|---:|---:|---:|"]
    for d in fast:
        lds = d.get("SQ_INSTS_LDS", 0.0)
        bc = d.get("SQ_LDS_BANK_CONFLICT", 0.0)
        act = d.get("SQ_LDS_IDX_ACTIVE", 0.0)
        lines.append("| %d | %.2f | %.4g | %.2f | %.4g | %.3f | %.4f |" % (
            d["cls"], d["ns"] / 1e6, lds, 100.0 * lds / max(1.0, d.get("SQ_INSTS_VALU", 0.0)), bc,
            bc / max(1.0, lds), bc / max(1.0, act)))
    lines += ["", "Over the pass:", "",
              "- lds_lane_instructions_per_cell: %.4f" % (64.0 * tot["SQ_INSTS_LDS"] / cells),
              "- lds_per_100_valu: %.3f" % (100.0 * tot["SQ_INSTS_LDS"] / max(1.0, tot["SQ_INSTS_VALU"])),
              "- bank_conflict_cycles_per_lds_instruction: %.4f"
              % (tot["SQ_LDS_BANK_CONFLICT"] / max(1.0, tot["SQ_INSTS_LDS"])),
              "- bank_conflict_share_of_lds_busy_cycles: %.5f"
              % (tot["SQ_LDS_BANK_CONFLICT"] / max(1.0, tot["SQ_LDS_IDX_ACTIVE"])),
              "- lds_busy_cycles_per_cu_busy_cycle: %.5f"
              % (tot["SQ_LDS_IDX_ACTIVE"] / max(1.0, tot["SQ_BUSY_CU_CYCLES"])),
              "- bank_conflict_cycles_per_cu_busy_cycle: %.6f"
              % (tot["SQ_LDS_BANK_CONFLICT"] / max(1.0, tot["SQ_BUSY_CU_CYCLES"])),
              "- sources_sha256: %s" % sources_digest(), ""]
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


LONG_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_WAVES", "SQ_WAVE_CYCLES",
                 "SQ_BUSY_CU_CYCLES", "SQ_WAIT_ANY", "GRBM_GUI_ACTIVE")
LONG_COUNTERS_PROFILE = os.path.join(ROOT, "profiles", "long_kernels_counters.md")


def summarize_long_counters(pmc_csv, sweep_json, out_path, commands):
    """Writes the instruction-count profile of the long-pair kernels from one
    rocprofv3 --pmc run of `bench.py --sweep` over the lengths it names (the
    JSON line gives each length's cells).  For each length and precision the
    counters of the timed passes' long-kernel dispatches are averaged per
    pass; VALU per CU-clock = SQ_INSTS_VALU / SQ_BUSY_CU_CYCLES, resident waves
    per SIMD = SQ_WAVE_CYCLES / SQ_BUSY_CU_CYCLES (calibrated on the general
    FP64 long kernel, which holds exactly one wave per SIMD and read 1.00)."""
    rec = None
    with open(sweep_json) as fh:
        for line in fh:
            if line.startswith("{"):
                rec = json.loads(line)
    rows = rec["sweep"]
    by = {}
    with open(pmc_csv, newline="") as fh:
        for r in csv.DictReader(fh):
            m = re.search(r"long_kernel<(float|double), (?:true|false)>", r["Kernel_Name"])
            if not m:
                continue
            d = by.setdefault(int(r["Dispatch_Id"]), dict(
                prec="fp32" if m.group(1) == "float" else "fp64",
                ns=int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    disp = [by[i] for i in sorted(by)]
    # dispatches in sweep order: per length, the FP32 mode's passes, then the
    # FP64 mode's; each pass launches the lean and the general long kernel of
    # both precisions (those of the other precision have no pairs), so per
    # length and precision the first passes are the FP32 mode's and the next
    # the FP64 mode's; a pass's lean and general dispatch are summed

    def per_pass(ds):
        out = []
        for k in range(0, len(ds) - 1, 2):
            a, b = ds[k], ds[k + 1]
            d = {c: a.get(c, 0.0) + b.get(c, 0.0) for c in set(a) | set(b) if c != "prec"}
            d["prec"] = a["prec"]
            out.append(d)
        return out
    f32 = per_pass([d for d in disp if d["prec"] == "fp32"])
    f64 = per_pass([d for d in disp if d["prec"] == "fp64"])
    lines = ["# Instruction counts of the long-pair kernels, equal-length pairs", "",
             "Commands (repository root, one MI355X):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", "Workload: the length sweep's batches (one read of L bases against 16 haplotypes"
              " of L bases per region); counters per pass of `long_kernel<float, *>` (FP32 mode) and"
              " `long_kernel<double, *>` (FP64 mode), the lean and the general kernel of the"
              " precision summed (the sweep's reads have one gap byte: all pairs run in the lean"
              " kernel), averaged over the passes of the run.", "",
              "| L | kernel | pairs | tiles/pair | ms | GCUPS | VALU per cell | SALU per cell |"
              " LDS per cell | VALU per CU-clock | waves per SIMD | wait share | clock GHz |",
              "|---:|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    per = {}
    n_pass = 1 + int(rec.get("reps", 1))
    for li, row in enumerate(rows):
        for mode in ("fp32", "fp64"):
            src, first = (f32, 2 * li * n_pass) if mode == "fp32" else (f64, (2 * li + 1) * n_pass)
            ds = src[first:first + n_pass]
            if not ds:
                continue
            t = {c: sum(d.get(c, 0.0) for d in ds) / len(ds) for c in LONG_COUNTERS}
            ns = sum(d["ns"] for d in ds) / len(ds)
            cells = row["cells"]
            busy = max(1.0, t["SQ_BUSY_CU_CYCLES"])
            per[(row["length"], mode)] = t
            lines.append("| %d | %s | %d | %d | %.2f | %.0f | %.2f | %.3f | %.3f | %.3f | %.2f | %.2f | %.2f |" % (
                row["length"], ds[0]["prec"], row["pairs"], -(-row["length"] // 1024), ns / 1e6,
                cells / ns, 64.0 * t["SQ_INSTS_VALU"] / cells, 64.0 * t["SQ_INSTS_SALU"] / cells,
                64.0 * t["SQ_INSTS_LDS"] / cells, t["SQ_INSTS_VALU"] / busy,
                t["SQ_WAVE_CYCLES"] / busy, t["SQ_WAIT_ANY"] / max(1.0, t["SQ_WAVE_CYCLES"]),
                t["GRBM_GUI_ACTIVE"] / 8.0 / max(1.0, ns)))
    lines += ["", "VALU, SALU and LDS are lane-instructions per useful cell (wave-instructions x 64 /"
              " cells); the wait share is SQ_WAIT_ANY / SQ_WAVE_CYCLES (wave-cycles spent waiting"
              " on anything).", "", "- sources_sha256: %s" % sources_digest(), ""]
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def summarize_trace(trace_csv, bench_json, out_path, commands):
    """Writes the kernel-duration profile of the FP32 short kernels from a
    rocprofv3 --kernel-trace run of bench.py: the forward passes on the whole
    batch (each 42 consecutive launches of `short_kernel<float, c, kind>`; the
    three with the largest total, i.e. not the autotuning passes on a
    sample), beside the HIP-event figure the same run printed."""
    rec = None
    with open(bench_json) as fh:
        for line in fh:
            if line.startswith("{"):
                rec = json.loads(line)
    if rec is None:
        raise SystemExit("no JSON line in %s" % bench_json)
    with open(trace_csv, newline="") as fh:
        rows = sorted(csv.DictReader(fh), key=lambda r: int(r["Start_Timestamp"]))
    calls, cur = [], []
    for r in rows:
        m = re.search(r"short_kernel<float, \d+, \d+>", r["Kernel_Name"])
        if not m:
            continue
        cur.append((m.group(0), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
        if len(cur) == 2 * N_CLASSES:
            calls.append(cur)
            cur = []
    n_big = rec["warmup"] + rec["steps"]
    tot = [sum(d for _, d in c) for c in calls]
    big = sorted(sorted(range(len(calls)), key=lambda i: -tot[i])[:n_big])
    per = {}
    for i in big:
        for name, d in calls[i]:
            a = per.setdefault(name, [0, 0.0])
            a[0] += 1
            a[1] += d
    steps_ms = [tot[i] / 1e3 for i in big]
    timed = steps_ms[rec["warmup"]:]
    cfg = rec["config"]
    lines = ["# Kernel durations of the FP32 short-pair kernels, genome-scale WGS-like batch", "",
             "Commands (repository root, one MI355X):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", "Workload: %d regions, %d pairs, %.6g cells. The run autotunes the pack costs on a"
              " sample before its timed steps, so the table is taken from the kernel trace"
              " (`run_kernel_trace.csv`): the %d forward calls on the whole batch (%d warm-up + %d"
              " timed), each 42 launches of `short_kernel<float, c, kind>` (class c has N = 4 + c"
              " columns per lane; kind 0 is the fast FP32 kernel, 1 the general one)."
              % (cfg["regions"], cfg["pairs"], cfg["cells"], n_big, rec["warmup"], rec["steps"]), "",
              "| kernel | calls | total us | average us |", "|---|---:|---:|---:|"]
    for name, (c, d) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        lines.append("| %s | %d | %.1f | %.1f |" % (name, c, d, d / c))
    lines += ["", "FP32 short-pair family per forward call (sum of its 42 launches): "
              + ", ".join("%.1f ms" % x for x in steps_ms)
              + "; mean of the timed calls %.1f ms." % (sum(timed) / len(timed)),
              "HIP events on the launch stream in the same run (`roofline.kernel_ms`, mean of the"
              " timed steps): %.1f ms." % rec["roofline"]["kernel_ms"], "",
              "- trace_family_ms: %.3f" % (sum(timed) / len(timed)),
              "- events_family_ms: %.3f" % rec["roofline"]["kernel_ms"],
              "- sources_sha256: %s" % sources_digest(), ""]
    # the plain FP64 passes of the same run (its fp64_plain leg): groups of
    # 21 consecutive launches of short_kernel<double, c, 2>, the two with the
    # largest total (the FP32 steps also launch them, for their few reruns)
    calls64, cur = [], []
    for r in rows:
        m = re.search(r"short_kernel<double, (\d+), 2>", r["Kernel_Name"])
        if not m:
            continue
        cur.append((int(m.group(1)), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
        if len(cur) == N_CLASSES:
            calls64.append(cur)
            cur = []
    if rec.get("fp64_plain") and len(calls64) >= 2:
        tot64 = [sum(d for _, d in c) for c in calls64]
        big64 = sorted(range(len(calls64)), key=lambda i: -tot64[i])[:2]
        lines += ["## Plain FP64 passes of the same run", "",
                  "Each of the two plain FP64 forward calls (`fp64_plain`: 1 warm-up + 1 timed) is 21"
                  " launches of `short_kernel<double, c, 2>`; mean duration per class (the FP64"
                  " kernels' occupancy targets: 1 wave per SIMD as the compiler chooses for"
                  " N = 4-8, 3 for N = 9-15, 2 for N = 16-24; packed with the run's autotuned"
                  " cost table, %s)." % ("N + %g" % (rec["pack_costs"]["fp64"][0] - 4)
                                         if rec.get("pack_costs") else "the default"), "",
                  "| class c (N = 4 + c) | ms |", "|---:|---:|"]
        for c in range(N_CLASSES):
            ds = [d for i in big64 for cc, d in calls64[i] if cc == c]
            lines.append("| %d | %.2f |" % (c, sum(ds) / len(ds) / 1e3))
        lines += ["", "- fp64_family_ms: %.3f" % (sum(tot64[i] for i in big64) / 2 / 1e3),
                  "- fp64_plain_ms_per_step: %.3f" % rec["fp64_plain"]["ms_per_step"], ""]
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def stored_traffic(regions):
    """Bytes per step of the FP32 short-kernel family from the committed
    profile, or None if it was taken on other sources or another workload."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    vals = dict(re.findall(r"^- (\w+): (\S+)$", open(TRAFFIC_PROFILE).read(), flags=re.M))
    if vals.get("sources_sha256") != sources_digest() or int(vals.get("regions", -1)) != regions:
        return None
    return float(vals["traffic_bytes_per_step"])


def _percentiles(x):
    if len(x) == 0:
        return None
    x = np.asarray(x) * 1e3
    return dict(n=int(len(x)), p50_ms=round(float(np.percentile(x, 50)), 3),
                p99_ms=round(float(np.percentile(x, 99)), 3), max_ms=round(float(x.max()), 3))


def serve_leg(phmm, args):
    """The served request stream: regions of the mixed workload (95% short,
    5% long-read regions) arrive Poisson at a fixed rate; the server batches
    them continuously.  First the sustainable capacity is measured by
    submitting a block of regions at once, then one stream runs for
    args.serve_seconds at each fraction of that capacity in args.serve_loads
    (fresh regions for each stream).  The server runs with its defaults
    (long-read regions on a long lane whose grids are a quarter of the chip's,
    so short regions never wait behind them); the same measurement with the
    long lane on the whole chip (the throughput setting) follows, one stream
    of args.serve_compare_seconds at 0.8 x its own capacity."""
    gen_chunk = 2000
    cache = {}

    def region(i):
        c = i // gen_chunk
        if c not in cache:
            cache[c] = synth.generate("served_stream", c * gen_chunk, gen_chunk)
        return synth.region_slice(cache[c], i - c * gen_chunk)

    def run(opts, loads, seconds, first):
        with phmm.Server(**opts) as srv:
            # capacity: a block submitted at once
            n_cap = args.serve_capacity_regions
            regs = [region(first + i) for i in range(n_cap)]
            t0 = time.perf_counter()
            ts = [srv.submit(r) for r in regs]
            cap_cells = 0
            for t in ts:
                _, _, info = srv.wait(t)
                cap_cells += info["cells"]
            span = time.perf_counter() - t0
            cap_rps = n_cap / span
            log("serving capacity (%s): %d regions, %.3g cells in %.2f s -> %.1f regions/s, %.1f GCUPS"
                % (opts, n_cap, cap_cells, span, cap_rps, cap_cells / span / 1e9))
            del regs
            cache.clear()
            streams = []
            first += n_cap
            for si, load in enumerate(loads):
                streams.append(_serve_stream(srv, region, first, load, cap_rps,
                                             cap_cells / span, seconds, seed=4 + si))
                first += streams[-1]["regions"]
                cache.clear()
        return dict(capacity_regions_per_s=round(cap_rps, 2),
                    capacity_gcups=round(cap_cells / span / 1e9, 2), streams=streams), first

    opts = dict(lanes=args.serve_lanes, long_lanes=1, hbm_budget_bytes=args.serve_budget_gib << 30,
                short_cu_percent=args.serve_short_cu)
    main, first = run(opts, args.serve_loads, args.serve_seconds, 0)
    res = dict(arrival="poisson", capacity_regions_per_s=main["capacity_regions_per_s"],
               capacity_gcups=main["capacity_gcups"], streams=main["streams"],
               lanes=args.serve_lanes, long_lanes=1, short_cu_percent=args.serve_short_cu,
               long_read_min=512, long_grid_percent=25, budget_gib=args.serve_budget_gib)
    if args.serve_compare_seconds > 0:
        alt, _ = run(dict(opts, long_grid_percent=100), [0.8], args.serve_compare_seconds, first)
        res["throughput_setting"] = dict(long_grid_percent=100, **alt)
    return res


def _serve_stream(srv, region, first, load, cap_rps, cap_cps, seconds, seed):
    """One Poisson stream at load x capacity (all its regions generated
    before the clock starts); latency percentiles over all, short and long
    regions.  The load is set in cells: the arrival rate is load x the
    capacity's cells per second / the mean cells per region of the stream's
    own regions (5% of the regions carry 98% of the cells, so a rate in
    regions taken from the capacity block alone can offer far more or less
    work than the fraction says)."""
    import threading
    n_est = int(load * cap_rps * seconds * 1.5) + 100
    regs = [region(first + q) for q in range(n_est)]
    mean_cells = sum(synth.batch_cells(r) for r in regs) / n_est
    rate = load * cap_cps / mean_cells
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * seconds * 1.2) + 10))
    arrivals = arrivals[arrivals < seconds]
    n = len(arrivals)
    regs += [region(first + q) for q in range(n_est, n)]
    del regs[n:]
    tickets = [None] * n
    late = [0.0]
    st0 = srv.stats()

    def submitter():
        base = time.perf_counter()
        for q in range(n):
            r = regs[q]
            d = base + arrivals[q] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            else:
                late[0] = max(late[0], -d)
            tickets[q] = srv.submit(r)
    th = threading.Thread(target=submitter)
    ts0 = time.perf_counter()
    th.start()
    lat, lat_s, lat_l, cells = [], [], [], 0
    for q in range(n):
        while tickets[q] is None:
            time.sleep(0.0002)
        _, _, info = srv.wait(tickets[q])
        lat.append(info["latency_s"])
        (lat_l if info["is_long"] else lat_s).append(info["latency_s"])
        cells += info["cells"]
    th.join()
    wall = time.perf_counter() - ts0
    st = srv.stats()
    res = dict(load=load, rate_regions_per_s=round(rate, 2),
               offered_gcups=round(rate * mean_cells / 1e9, 2), seconds=seconds, regions=n,
               cells=cells, gcups=round(cells / wall / 1e9, 2),
               latency_all=_percentiles(lat), latency_short=_percentiles(lat_s),
               latency_long=_percentiles(lat_l),
               batches=int(st["batches"] - st0["batches"]),
               full_batches=int(st["full_batches"] - st0["full_batches"]),
               max_submit_lag_ms=round(late[0] * 1e3, 3), cu_mask_status=int(st["cu_mask_status"]))
    log("served stream at %.1fx capacity: %d regions at %.1f/s, p50 %.2f ms, p99 %.2f ms, %.1f GCUPS"
        % (load, n, rate, res["latency_all"]["p50_ms"], res["latency_all"]["p99_ms"], res["gcups"]))
    return res


def pair_cells(batch):
    rl = np.diff(batch["read_offsets"]).astype(np.int64)
    hl = np.diff(batch["hap_offsets"]).astype(np.int64)
    pl = batch["pair_list"]
    return rl[pl[:, 0]] * hl[pl[:, 1]], rl[pl[:, 0]], hl[pl[:, 1]]


class ClockSampler:
    """Samples the GPU's current shader clock (the starred level of the
    amdgpu kernel module's pp_dpm_sclk table in sysfs) every `period`
    seconds on a thread, between start() and stop(); summary() is None where
    the table cannot be read."""

    def __init__(self, period=0.25):
        import glob
        self.paths = sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"))
        self.period, self.samples, self._stop = period, [], None

    def _read(self):
        best = None
        for p in self.paths:
            try:
                with open(p) as fh:
                    for line in fh:
                        if "*" in line:
                            m = re.search(r"(\d+)\s*[Mm][Hh]z", line)
                            if m:
                                best = max(best or 0, int(m.group(1)))
            except OSError:
                pass
        return best

    def start(self):
        import threading
        self._stop = threading.Event()

        def run():
            while not self._stop.wait(self.period):
                v = self._read()
                if v:
                    self.samples.append(v)
        self._th = threading.Thread(target=run, daemon=True)
        self._th.start()
        return self

    def stop(self):
        self._stop.set()
        self._th.join()

    def summary(self):
        if not self.samples:
            return None
        x = np.array(self.samples)
        return dict(median=int(np.median(x)), min=int(x.min()), max=int(x.max()), samples=len(x),
                    source="pp_dpm_sclk (current level), every %.2f s of the timed steps"
                    % self.period)


def time_steps(phmm, torch, ctx, db, out, fl, ws, stream, warmup, steps, per_step=None):
    for i in range(warmup):
        phmm.phmm_forward_batch_async(ctx, db, out, fl, ws, stream)
        stream.synchronize()
        log("warmup step %d done" % (i + 1))
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for i in range(steps):
        phmm.phmm_forward_batch_async(ctx, db, out, fl, ws, stream)
        phases.append(phmm.phmm_last_timing(ctx))  # waits for this step's last event
        log("step %d: %.1f ms" % (i + 1, phases[-1]["total_ms"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    phmm.phmm_device_status(ctx, ws)
    avg = {k: float(np.mean([p[k] for p in phases])) for k in phases[0]}
    if per_step is not None:
        per_step.extend(p["total_ms"] for p in phases)
    return elapsed, avg


SWEEP_LENGTHS = (32, 64, 128, 256, 512, 1024, 1536, 2048, 4096, 8192, 16384, 32768, 65536,
                 131072)


def sweep_leg(phmm, torch, args):
    """Length sweep of equal-length pairs (read and haplotypes of L bases,
    16 haplotypes per read), L = 32 ... 131072: kernel-only GCUPS (HIP events
    around the whole pass, packer included) in the default FP32 + rerun mode
    and in plain FP64, best of `--sweep-reps` passes after one warm-up, from
    stream launches of the asynchronous call and from the synchronous call
    (whose pass launches only the kernels with work).  With
    `--sweep-long-fp32` the FP32 mode also runs long pairs in the FP32 long
    kernel (by default they run in FP64)."""
    rows = []
    for L in args.sweep_lengths or SWEEP_LENGTHS:
        regions = max(1, min(1_000_000, int(math.ceil(args.sweep_cells / (16.0 * L * L)))))
        b = synth.generate(synth.sweep_cfg(L, regions))
        cells = int(pair_cells(b)[0].sum())
        db = phmm.DeviceBatch(b, "cuda:0")
        n = len(b["pair_list"])
        out = torch.empty(n, dtype=torch.float64, device="cuda:0")
        fl = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        res = {"length": L, "regions": regions, "pairs": n, "cells": cells}
        for mode, prec, peak in (("fp32", phmm.PHMM_FP32_RERUN, FP32_PEAK_TFLOPS),
                                 ("fp64", phmm.PHMM_FP64_PLAIN, FP32_PEAK_TFLOPS / 2)):
            opts = dict(long_fp32_max_rows=131072) if (args.sweep_long_fp32 and
                                                        prec == phmm.PHMM_FP32_RERUN) else {}
            ctx = phmm.Context(precision=prec, timing=True, **opts)
            ws = torch.empty(phmm.phmm_workspace_bytes(ctx, n, db.max_read_len, db.max_hap_len),
                             dtype=torch.uint8, device="cuda:0")
            stream = torch.cuda.Stream()
            best = None
            for r in range(1 + args.sweep_reps):
                phmm.phmm_forward_batch_async(ctx, db, out, fl, ws, stream)
                t = phmm.phmm_last_timing(ctx)["total_ms"]
                if r > 0:
                    best = t if best is None else min(best, t)
            phmm.phmm_device_status(ctx, ws)
            f = fl.cpu().numpy()
            res[mode] = dict(ms=round(best, 3), gcups=round(cells / best / 1e6, 1),
                             roofline_frac=round(FLOPS_PER_CELL * cells / (best / 1e3) / (peak * 1e12), 4),
                             fp32_pairs=int(((f & 0x01) != 0).sum()), long_pairs=int(((f & 0x04) != 0).sum()),
                             rerun_pairs=int(((f & 0x02) != 0).sum()))
            # the synchronous call (host arrays): its pass launches only the
            # kernels with work; device time from its HIP events
            sb = None
            for r in range(1 + args.sweep_reps):
                phmm.phmm_forward_batch(ctx, b)
                t = phmm.phmm_last_timing(ctx)["total_ms"]
                if r > 0:
                    sb = t if sb is None else min(sb, t)
            res[mode]["sync_pass"] = dict(ms=round(sb, 3), gcups=round(cells / sb / 1e6, 1))
            ctx.close()
            del ws
        log("sweep L=%d: %d pairs, %.3g cells; FP32+rerun %.1f GCUPS (%.1f ms), FP64 %.1f GCUPS (%.1f ms)" %
            (L, n, cells, res["fp32"]["gcups"], res["fp32"]["ms"], res["fp64"]["gcups"], res["fp64"]["ms"]))
        rows.append(res)
        del db, out, fl
        torch.cuda.empty_cache()
    return rows


def _best_pass(phmm, torch, ctx, db, reps):
    """Best total of `reps` passes after one warm-up (HIP events), flags of the last."""
    n = db.n_pairs
    out = torch.empty(n, dtype=torch.float64, device="cuda:0")
    fl = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    ws = torch.empty(phmm.phmm_workspace_bytes(ctx, n, db.max_read_len, db.max_hap_len),
                     dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.Stream()
    best = None
    for r in range(1 + reps):
        phmm.phmm_forward_batch_async(ctx, db, out, fl, ws, stream)
        t = phmm.phmm_last_timing(ctx)["total_ms"]
        if r > 0:
            best = t if best is None else min(best, t)
    phmm.phmm_device_status(ctx, ws)
    return best, fl.cpu().numpy()


def _best_graph(phmm, torch, ctx, db, reps):
    """Best of `reps` replays of the pass from the context's captured HIP
    graph after one warm-up (which captures it), timed by events around the
    call on its stream."""
    n = db.n_pairs
    out = torch.empty(n, dtype=torch.float64, device="cuda:0")
    fl = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    ws = torch.empty(phmm.phmm_workspace_bytes(ctx, n, db.max_read_len, db.max_hap_len),
                     dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.Stream()
    best = None
    for r in range(1 + reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        phmm.phmm_forward_batch_graph(ctx, db, out, fl, ws, stream)
        e1.record(stream)
        stream.synchronize()
        if r > 0:
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
    phmm.phmm_device_status(ctx, ws)
    return best


def batched_uneven_leg(phmm, torch, args):
    """The batched uneven short-pair workload (20,000 regions, 2-8 variant
    haplotypes of 150-600 bp, 100-150 bp reads) and its stress variant with
    i.i.d. haplotypes, in FP32 + rerun and in plain FP64: kernel-only GCUPS
    and the share of pairs rerun in FP64; the FP32 + rerun pass also replayed
    from its captured HIP graph, and both modes through the synchronous call
    (device time of its pass)."""
    res = {}
    for name, cfg in (("variant_haplotypes", "batched_uneven"), ("iid_haplotypes", synth.iid_haps_cfg("batched_uneven"))):
        b = synth.generate(cfg)
        cells = int(pair_cells(b)[0].sum())
        db = phmm.DeviceBatch(b, "cuda:0")
        r = {"pairs": db.n_pairs, "cells": cells}
        for mode, prec in (("fp32_rerun", phmm.PHMM_FP32_RERUN), ("fp64", phmm.PHMM_FP64_PLAIN)):
            with phmm.Context(precision=prec, timing=True) as ctx:
                ms, f = _best_pass(phmm, torch, ctx, db, args.small_reps // 10 or 1)
            r[mode] = dict(ms=round(ms, 3), gcups=round(cells / ms / 1e6, 1))
            if prec == phmm.PHMM_FP32_RERUN:
                r["rerun_fraction"] = round(float(((f & 0x02) != 0).mean()), 4)
                with phmm.Context(precision=prec) as gctx:
                    gms = _best_graph(phmm, torch, gctx, db, args.small_reps // 10 or 1)
                r["fp32_rerun_graph"] = dict(ms=round(gms, 3), gcups=round(cells / gms / 1e6, 1))
        r["speedup_fp32_rerun"] = round(r["fp64"]["ms"] / r["fp32_rerun"]["ms"], 3)
        # the synchronous call's pass (host arrays; device time from its HIP
        # events), which launches only the kernels that have work
        sync = {}
        for mode, prec in (("fp32_rerun", phmm.PHMM_FP32_RERUN), ("fp64", phmm.PHMM_FP64_PLAIN)):
            with phmm.Context(precision=prec, timing=True) as ctx:
                ts = []
                for rep in range(3):
                    phmm.phmm_forward_batch(ctx, b)
                    ts.append(phmm.phmm_last_timing(ctx)["total_ms"])
            ms = min(ts[1:])
            sync[mode] = dict(ms=round(ms, 3), gcups=round(cells / ms / 1e6, 1))
        r["sync_pass"] = sync
        log("batched uneven pairs (%s): %d pairs, %.3g cells; FP32+rerun %.1f GCUPS (rerun %.1f%%), "
            "FP64 %.1f GCUPS" % (name, r["pairs"], cells, r["fp32_rerun"]["gcups"],
                                100 * r["rerun_fraction"], r["fp64"]["gcups"]))
        res[name] = r
        del db
        torch.cuda.empty_cache()
    return res


def one_pair_per_wave_leg(phmm, torch, args, costs):
    """FP64 on the first `args.opw_regions` regions of the genome-scale
    workload in two forms: one pair per wavefront (no packing) and packed as
    the FP64 path runs it, beside FP32 + rerun on the same pairs."""
    b = synth.generate("genome_scale", 0, args.opw_regions)
    cells = int(pair_cells(b)[0].sum())
    db = phmm.DeviceBatch(b, "cuda:0")
    res = {"regions": args.opw_regions, "pairs": db.n_pairs, "cells": cells}
    for name, kw in (("fp64_one_pair_per_wave", dict(precision=phmm.PHMM_FP64_PLAIN,
                                                      one_pair_per_wave=True)),
                     ("fp64_packed", dict(precision=phmm.PHMM_FP64_PLAIN)),
                     ("fp32_rerun_packed", dict(precision=phmm.PHMM_FP32_RERUN))):
        with phmm.Context(timing=True, **kw) as ctx:
            if costs is not None:
                ctx.set_class_costs(costs)
            ms, _ = _best_pass(phmm, torch, ctx, db, 1)
        res[name] = dict(ms=round(ms, 3), gcups=round(cells / ms / 1e6, 1))
    log("FP64 one pair per wave %.1f GCUPS, FP64 packed %.1f, FP32+rerun packed %.1f (%d regions)"
        % (res["fp64_one_pair_per_wave"]["gcups"], res["fp64_packed"]["gcups"],
           res["fp32_rerun_packed"]["gcups"], args.opw_regions))
    del db
    torch.cuda.empty_cache()
    return res


LONG_GOLDEN = os.path.join(ROOT, "tests", "golden", "long_reads_all.json")


def long_reads_leg(phmm, torch, args):
    """The long-read workload: 96 pairs, 32 each of 10,000, 32,000 and 100,000
    base reads against haplotypes 1.1 times as long (5% substitutions, 2%
    indels of 1-10 bp, Phred 5-30, ins/del 30, gcp 10), one pass over all of
    them and one per length class: kernel-only GCUPS (HIP events, best of
    `--long-reps` after a warm-up), the fraction of the vector roofline of
    the precision each class runs in, and every result's error against the
    oracle values stored by tests/golden/make_long_reads_all.py.  Twice: with
    the library's defaults (every long pair in the FP64 long kernel) and with
    the FP32 long kernel enabled for every read length (long_fp32_max_rows =
    PHMM_MAX_READ; exact enough on this workload, not for every input)."""
    with open(LONG_GOLDEN) as fh:
        gold = json.load(fh)["pairs"]
    want = np.array([float(g["log10_l"]) for g in gold])
    b = synth.generate("long_reads")
    cells_pp, rl, hl = pair_cells(b)
    assert np.array_equal(rl, [g["read_len"] for g in gold]) and \
        np.array_equal(hl, [g["hap_len"] for g in gold])

    def one_pass(bb, cells, opts):
        db = phmm.DeviceBatch(bb, "cuda:0")
        n = db.n_pairs
        out = torch.empty(n, dtype=torch.float64, device="cuda:0")
        fl = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        with phmm.Context(timing=True, **opts) as ctx:
            ws = torch.empty(phmm.phmm_workspace_bytes(ctx, n, db.max_read_len, db.max_hap_len),
                             dtype=torch.uint8, device="cuda:0")
            stream = torch.cuda.Stream()
            best = None
            for r in range(1 + args.long_reps):
                phmm.phmm_forward_batch_async(ctx, db, out, fl, ws, stream)
                t = phmm.phmm_last_timing(ctx)["total_ms"]
                if r > 0:
                    best = t if best is None else min(best, t)
            phmm.phmm_device_status(ctx, ws)
        return best, out.cpu().numpy(), fl.cpu().numpy()

    def run(opts, label):
        res = {"pairs": len(gold), "cells": int(cells_pp.sum())}
        ms, got, f = one_pass(b, res["cells"], opts)
        res["all"] = dict(ms=round(ms, 2), gcups=round(res["cells"] / ms / 1e6, 1))
        classes = []
        for L in (10000, 32000, 100000):
            idx = np.nonzero(rl == L)[0]
            sub = synth.subset_pairs(b, idx)
            c = int(cells_pp[idx].sum())
            cms, cgot, cf = one_pass(sub, c, opts)
            fp32 = bool(np.all(cf & 0x01))
            peak = FP32_PEAK_TFLOPS if fp32 else FP32_PEAK_TFLOPS / 2
            err = np.abs(got[idx] - want[idx])
            classes.append(dict(read_len=L, pairs=len(idx), cells=c, ms=round(cms, 2),
                                gcups=round(c / cms / 1e6, 1), precision="fp32" if fp32 else "fp64",
                                roofline_frac=round(FLOPS_PER_CELL * c / (cms / 1e3) / (peak * 1e12), 4),
                                max_err=float(err.max()), mean_err=float(err.mean()),
                                bound=1e-4 if fp32 else 1e-10,
                                ok=bool(err.max() <= (1e-4 if fp32 else 1e-10)),
                                flags=sorted(set(int(x) for x in f[idx]))))
            log("long reads (%s) %d bp: %d pairs, %.1f GCUPS (%s, %.1f%% of its roofline), max err %.3g"
                % (label, L, len(idx), classes[-1]["gcups"], classes[-1]["precision"],
                   100 * classes[-1]["roofline_frac"], classes[-1]["max_err"]))
        res["classes"] = classes
        res["ok"] = all(c["ok"] for c in classes)
        log("long-read workload (%s): %d pairs, %.3g cells, %.1f GCUPS in one pass"
            % (label, res["pairs"], res["cells"], res["all"]["gcups"]))
        return res

    res = run({}, "defaults: FP64 long kernel")
    res["fp32_long_kernel"] = run(dict(long_fp32_max_rows=131072), "FP32 long kernel enabled")
    torch.cuda.empty_cache()
    return res


def small_batch_leg(phmm, torch, args):
    """Latency of one small batch (about 3550 short pairs, all at once): the
    whole pass on device-resident inputs (HIP events, packer included), and
    the synchronous host-to-host call (inputs copied in, results copied
    back), median and minimum over `--small-reps` calls after warm-up."""
    b = synth.generate(synth.small_batch_cfg())
    cells = int(pair_cells(b)[0].sum())
    n = len(b["pair_list"])
    db = phmm.DeviceBatch(b, "cuda:0")
    out = torch.empty(n, dtype=torch.float64, device="cuda:0")
    fl = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    res = {"pairs": n, "cells": cells}
    with phmm.Context(timing=True) as ctx:
        ws = torch.empty(phmm.phmm_workspace_bytes(ctx, n, db.max_read_len, db.max_hap_len),
                         dtype=torch.uint8, device="cuda:0")
        stream = torch.cuda.Stream()
        dev, phases = [], []
        for r in range(5 + args.small_reps):
            phmm.phmm_forward_batch_async(ctx, db, out, fl, ws, stream)
            t = phmm.phmm_last_timing(ctx)
            if r >= 5:
                dev.append(t["total_ms"])
                phases.append(t)
        phmm.phmm_device_status(ctx, ws)
        # the same pass from stream launches and replayed from the context's
        # captured HIP graph, both timed by events around the call on the
        # stream (device) and by the host clock from the call to the end of
        # a stream synchronisation (submission included)
        launch = {}
        for how, fn in (("stream_launches", phmm.phmm_forward_batch_async),
                        ("graph_replay", phmm.phmm_forward_batch_graph)):
            evs, walls = [], []
            for r in range(5 + args.small_reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                t0 = time.perf_counter()
                e0.record(stream)
                fn(ctx, db, out, fl, ws, stream)
                e1.record(stream)
                stream.synchronize()
                if r >= 5:
                    walls.append((time.perf_counter() - t0) * 1e3)
                    evs.append(e0.elapsed_time(e1))
            launch[how] = dict(device_ms_median=round(float(np.median(evs)), 4),
                               device_ms_min=round(min(evs), 4),
                               call_to_done_ms_median=round(float(np.median(walls)), 4))
        res["launch"] = launch
        host, sync = [], []
        for r in range(5 + args.small_reps):
            t0 = time.perf_counter()
            phmm.phmm_forward_batch(ctx, b)
            if r >= 5:
                host.append((time.perf_counter() - t0) * 1e3)
                sync.append(phmm.phmm_last_timing(ctx)["total_ms"])
    ph = {k: round(float(np.median([p[k] for p in phases])), 4) for k in phases[0]}
    res.update(device_ms_median=round(float(np.median(dev)), 4), device_ms_min=round(min(dev), 4),
               sync_pass_ms_median=round(float(np.median(sync)), 4),
               host_to_host_ms_median=round(float(np.median(host)), 4),
               host_to_host_ms_min=round(min(host), 4), phases_ms_median=ph)
    log("small batch: stream launches %s, graph replay %s" % (res["launch"]["stream_launches"],
                                                               res["launch"]["graph_replay"]))
    log("small batch: %d pairs, %.3g cells: asynchronous pass %.3f ms (min %.3f), synchronising "
        "pass %.3f ms, host-to-host %.3f ms; asynchronous phases %s"
        % (n, cells, res["device_ms_median"], res["device_ms_min"], res["sync_pass_ms_median"],
           res["host_to_host_ms_median"], ph))
    return res


def cpu_rowform_leg(batch, sidx, scells, ovals, cores):
    """The CPU comparator (row-level formulation, SIMD rows, threads over
    pairs) on the oracle's sample: best of two runs, error against the
    oracle."""
    import cpu_rowform
    walls = []
    for _ in range(2):
        t = time.perf_counter()
        vals, flags = cpu_rowform.forward_pairs(batch, sidx, threads=cores)
        walls.append(time.perf_counter() - t)
    wall = min(walls)
    fin = np.isfinite(ovals)
    d = np.abs(np.where(fin, vals, 0.0) - np.where(fin, ovals, 0.0))
    res = dict(value=round(scells / wall / 1e9, 3), unit="GCUPS", cores=cores,
               kind="row-level formulation on the host (AVX2 rows, OpenMP over pairs, FP32 "
                    "with FP64 rerun)", seconds=round(wall, 3),
               fp64_pairs=int((flags == 2).sum()),
               max_err_fp32=float(d[flags == 1].max(initial=0.0)),
               max_err_fp64=float(d[flags == 2].max(initial=0.0)))
    log("CPU row-form comparator: %.3f GCUPS on %d threads" % (res["value"], cores))
    return res


def genotype_leg(phmm, torch, ctx, batch, out, stream, reps):
    """Genotype likelihoods of every region of the step, straight on the
    forward pass's device output (phmm_genotype_batch_async): kernel time
    from HIP events on its stream, best of reps after a warm-up."""
    rp, rr, rh = batch["region_pairs"], batch["region_reads"], batch["region_haps"]
    R = np.diff(rr).astype(np.int64)
    H = np.diff(rh).astype(np.int64)
    go, n_gl = phmm.genotype_offsets(H)
    dev = "cuda:0"
    lo_d = torch.from_numpy(rp[:-1].astype(np.int64)).to(dev)
    r_d = torch.from_numpy(R.astype(np.int32)).to(dev)
    h_d = torch.from_numpy(H.astype(np.int32)).to(dev)
    go_d = torch.from_numpy(go.astype(np.int64)).to(dev)
    gl = torch.empty(n_gl, dtype=torch.float64, device=dev)
    best = torch.empty(len(H), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    times = []
    for r in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            phmm.phmm_genotype_batch_async(ctx, out, lo_d, r_d, h_d, go_d, gl, best, stream)
            e1.record(stream)
        e1.synchronize()
        if r > 0:
            times.append(e0.elapsed_time(e1))
    ms = min(times)
    gl_h = gl.cpu().numpy()
    G = H * (H + 1) // 2
    terms = int((G * R).sum())
    het = int(((G - H) * R).sum())
    nbytes = 8 * int((R * H).sum()) + 8 * n_gl + 4 * len(H) + 24 * len(H)
    log("genotype likelihoods: %d regions, %.3g read terms (%.3g heterozygous) in %.3f ms"
        % (len(H), terms, het, ms))
    return gl_h, dict(ms=round(ms, 3), regions=len(H), genotypes=n_gl, read_terms=terms,
                het_read_terms=het, g_terms_per_s=round(terms / (ms * 1e-3) / 1e9, 2),
                gb_per_s=round(nbytes / (ms * 1e-3) / 1e9, 1),
                note="diploid genotype log10-likelihoods of every region from the step's "
                     "log10 P(read|hap) on the device; FP64: a power per read and haplotype, "
                     "a multiply and frexp per read and genotype, a logarithm per genotype")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--regions", type=int, default=1000000,
                    help="regions of the workload (default: all 1,000,000)")
    ap.add_argument("--cpu-regions", type=int, default=1500,
                    help="regions in the oracle sample (CPU baseline and sampled parity)")
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="timed steps of the plain FP64 path on the same batch (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--end-to-end", type=int, default=1,
                    help="time the synchronous host-to-host call on the whole batch (0 = skip)")
    ap.add_argument("--opw-regions", type=int, default=20000,
                    help="regions for the FP64 one-pair-per-wave comparison (0 = skip)")
    ap.add_argument("--uneven", type=int, default=1,
                    help="run the batched uneven short-pair workload and its i.i.d. stress "
                         "variant (0 = skip)")
    ap.add_argument("--genotype-reps", type=int, default=3,
                    help="timed runs of the genotype-likelihood kernel on the step's output "
                         "(0 skips it)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default pack cost model instead of measuring it")
    ap.add_argument("--long-reps", type=int, default=2,
                    help="timed passes of the long-read leg (0: skip the leg)")
    ap.add_argument("--long-reads", action="store_true",
                    help="print only the long-read leg")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the served Poisson stream (0 = no serving leg)")
    ap.add_argument("--serve-compare-seconds", type=float, default=20.0,
                    help="served stream with the long lane on the whole chip (0 = skip)")
    ap.add_argument("--serve-loads", type=lambda v: [float(x) for x in v.split(",")],
                    default=[0.5, 0.8],
                    help="arrival rates of the streams as fractions of the measured serving "
                         "capacity (comma-separated)")
    ap.add_argument("--serve-capacity-regions", type=int, default=3000)
    ap.add_argument("--serve-lanes", type=int, default=3)
    ap.add_argument("--serve-budget-gib", type=int, default=24)
    ap.add_argument("--serve-short-cu", type=int, default=0,
                    help="percent of CUs for the short lanes (0 = no CU masks)")
    ap.add_argument("--calib-copy-mib", type=int, default=1024,
                    help="size of the calibration copy run before the timed steps")
    ap.add_argument("--sweep", action="store_true",
                    help="run only the length sweep of equal-length pairs (32 .. 131072) and "
                         "print its JSON line")
    ap.add_argument("--sweep-cells", type=float, default=1e11,
                    help="cells per length in the sweep (capped at 1,000,000 regions)")
    ap.add_argument("--sweep-reps", type=int, default=3)
    ap.add_argument("--sweep-long-fp32", action="store_true",
                    help="sweep: FP32 mode runs long pairs in the FP32 long kernel")
    ap.add_argument("--sweep-lengths", type=lambda v: [int(x) for x in v.split(",")], default=None,
                    help="comma-separated lengths of the sweep (default: 32 ... 131072)")
    ap.add_argument("--summarize-long-counters", nargs=2, metavar=("PMC_CSV", "SWEEP_JSON"),
                    help="write profiles/long_kernels_counters.md from a --pmc run of --sweep")
    ap.add_argument("--small-batch", action="store_true",
                    help="run only the small-batch latency leg (about 3550 short pairs)")
    ap.add_argument("--small-reps", type=int, default=50,
                    help="calls timed in the small-batch leg (0 = skip it in the default run)")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic profile from two rocprofv3 --pmc runs (no GPU used)")
    ap.add_argument("--summarize-lds", nargs=2, metavar=("PMC_CSV", "BENCH_JSON"),
                    help="write the LDS profile from a rocprofv3 --pmc run with the LDS counters")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("PMC_CSV", "BENCH_JSON"),
                    help="write the VALU counter profile from a rocprofv3 --pmc run with "
                         + " ".join(VALU_COUNTERS) + " and its bench.py output (no GPU used)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_CSV", "BENCH_JSON"),
                    help="write the kernel-duration profile from a rocprofv3 --kernel-trace run "
                         "and its bench.py output (no GPU used)")
    ap.add_argument("--command", action="append", default=[],
                    help="with --summarize-traffic: a command line to record in the profile")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace[0], args.summarize_trace[1], TRACE_PROFILE,
                        args.command)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters[0], args.summarize_counters[1], COUNTERS_PROFILE,
                           args.command)
        return
    if args.summarize_lds:
        summarize_lds(args.summarize_lds[0], args.summarize_lds[1], LDS_PROFILE, args.command)
        return
    if args.summarize_long_counters:
        summarize_long_counters(args.summarize_long_counters[0], args.summarize_long_counters[1],
                                LONG_COUNTERS_PROFILE, args.command)
        return
    if args.summarize_traffic:
        summarize_traffic(args.summarize_traffic[0], args.summarize_traffic[1], TRAFFIC_PROFILE,
                          args.regions, args.calib_copy_mib, args.command)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only; this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.small_batch:
        import torch
        import paper_2606_25738_amd as phmm
        print(json.dumps({"small_batch": small_batch_leg(phmm, torch, args), "data": "synthetic"}))
        return
    if args.long_reads:
        import torch
        import paper_2606_25738_amd as phmm
        print(json.dumps({"long_reads": long_reads_leg(phmm, torch, args), "data": "synthetic"}))
        return
    if args.sweep:
        import torch
        import paper_2606_25738_amd as phmm
        rows = sweep_leg(phmm, torch, args)
        print(json.dumps({"sweep": rows, "unit": "GCUPS (kernel-only)", "data": "synthetic",
                          "reps": args.sweep_reps, "long_fp32": bool(args.sweep_long_fp32),
                          "workload": "equal-length pairs, 16 haplotypes per read"}))
        return

    t = time.perf_counter()
    batch = synth.generate("genome_scale", 0, args.regions)
    cells_pp, rl, hl = pair_cells(batch)
    cells = int(cells_pp.sum())
    n_pairs = len(cells_pp)
    log("generated %d regions, %d pairs, %.4g cells in %.1fs"
        % (args.regions, n_pairs, cells, time.perf_counter() - t))

    # oracle sample first: worker processes fork before the GPU is touched
    cores = min(16, os.cpu_count() or 1)
    cpu = None
    rowform = None
    if not args.no_cpu and args.cpu_regions > 0:
        sidx, nreg = sample_pairs(batch, args.cpu_regions)
        scells = int(cells_pp[sidx].sum())
        log("oracle on %d pairs (%d regions, %.3g cells), %d processes" % (len(sidx), nreg, scells, cores))
        ovals, wall, cpusec = run_oracle(batch, sidx, cores)
        ncpu, naff = _host_cpus()
        cpu = dict(value=round(scells / wall / 1e9, 4), unit="GCUPS", cores=cores, kind="oracle",
                   cpu_model=_cpu_model(), host_logical_cpus=ncpu, affinity_cpus=naff,
                   cores_note="one single-threaded oracle process per logical CPU this process "
                              "may run on, at most 16",
                   single_core_gcups=round(scells / cpusec / 1e9, 4),
                   sample="%d random regions of the same workload (%d pairs, %.3g cells); "
                          "single-core %.3f GCUPS" % (nreg, len(sidx), scells,
                                                       scells / cpusec / 1e9),
                   seconds=round(wall, 2))
        log("oracle %.1fs wall, %.3f GCUPS on %d processes" % (wall, cpu["value"], cores))
        rowform = cpu_rowform_leg(batch, sidx, scells, ovals, cores)

    import torch
    import paper_2606_25738_amd as phmm

    t = time.perf_counter()
    db = phmm.DeviceBatch(batch, "cuda:0")
    torch.cuda.synchronize()
    log("inputs resident in HBM (%.1fs)" % (time.perf_counter() - t))
    stream = torch.cuda.Stream()
    out = torch.empty(n_pairs, dtype=torch.float64, device="cuda:0")
    fl = torch.empty(n_pairs, dtype=torch.uint8, device="cuda:0")

    peak32, peak64 = phmm.phmm_vector_peak(0)
    log("measured vector FMA peak: FP32 %.1f TFLOP/s, FP64 %.1f TFLOP/s" % (peak32, peak64))
    ctx = phmm.Context(timing=True)
    costs = None
    if not args.no_autotune:
        # the cost table (N + a, a from a fixed set, or the default N + 3)
        # that runs a sample of this workload (its first 50,000 regions)
        # fastest
        t = time.perf_counter()
        ns = min(args.regions, 50000)
        sb = synth.generate("genome_scale", 0, ns)
        sdb = phmm.DeviceBatch(sb, "cuda:0")
        sws = torch.empty(phmm.phmm_workspace_bytes(ctx, len(sb["pair_list"]), sdb.max_read_len,
                                                    sdb.max_hap_len), dtype=torch.uint8, device="cuda:0")
        costs = ctx.autotune_sample(sdb, sws, stream)
        del sdb, sws, sb
        log("autotuned pack costs in %.2fs (FP32 table): %s"
            % (time.perf_counter() - t, np.round(costs[0], 2).tolist()))
    ws = torch.empty(phmm.phmm_workspace_bytes(ctx, n_pairs, db.max_read_len, db.max_hap_len),
                     dtype=torch.uint8, device="cuda:0")
    copy_gbs = None
    if args.calib_copy_mib > 0:
        # plain copy of known size: the reference for the traffic counters
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            phmm.phmm_copy_calib(src, dst, stream)
            e1.record(stream)
        e1.synchronize()
        copy_gbs = 2.0 * nb / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del src, dst
        log("calibration copy: %d MiB, %.0f GB/s" % (args.calib_copy_mib, copy_gbs))
    step_ms = []
    clock = ClockSampler().start()
    try:
        elapsed, ph = time_steps(phmm, torch, ctx, db, out, fl, ws, stream, args.warmup,
                                 args.steps, step_ms)
    finally:
        clock.stop()
    counts = phmm.phmm_last_counts(ctx, ws)
    ms_per_step = elapsed * 1000.0 / args.steps
    value = cells / (elapsed / args.steps) / 1e9
    out_h = out.cpu().numpy()
    fl_h = fl.cpu().numpy()

    # dominant kernel: the FP32 short-pair kernels (one launch per column class)
    short = (hl <= 64 * 24)
    cells32 = int(cells_pp[short].sum())
    # algorithmic HBM bytes of the short pairs, per pair: the five per-base read
    # arrays, the haplotype, and 9 output bytes (log10 L and the flag)
    alg_bytes = float((5 * rl[short] + hl[short] + 9).sum())
    achieved = FLOPS_PER_CELL * cells32 / (ph["short_ms"] / 1e3) / 1e12
    traffic = stored_traffic(args.regions)
    roof = dict(bound="alu", achieved=round(achieved, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                frac=round(achieved / FP32_PEAK_TFLOPS, 4),
                traffic=None if traffic is None else round(traffic),
                traffic_unit="bytes per step (42 launches)",
                algorithmic_bytes=int(alg_bytes), hbm_gbs_from_traffic=None if traffic is None
                else round(traffic / (ph["short_ms"] / 1e3) / 1e9, 2), copy_calib_gbs=copy_gbs,
                kernel="FP32 short-pair kernels (fast and general kernel of each of the 21 column "
                       "classes: 42 launches per step)",
                kernel_ms=round(ph["short_ms"], 3),
                measured_peak_fp32=round(peak32, 2), measured_peak_fp64=round(peak64, 2),
                frac_of_measured=round(achieved / peak32, 4))

    fp64 = None
    if args.fp64_steps > 0:
        ctx64 = phmm.Context(precision=phmm.PHMM_FP64_PLAIN, timing=True)
        if costs is not None:
            ctx64.set_class_costs(costs)
        out64 = torch.empty_like(out)
        fl64 = torch.empty_like(fl)
        e64, ph64 = time_steps(phmm, torch, ctx64, db, out64, fl64, ws, stream, 1, args.fp64_steps)
        fp64 = dict(gcups=round(cells / (e64 / args.fp64_steps) / 1e9, 2),
                    ms_per_step=round(e64 * 1000 / args.fp64_steps, 2),
                    speedup_fp32_rerun=round(value / (cells / (e64 / args.fp64_steps) / 1e9), 3))
        ctx64.close()

    genotype = None
    if args.genotype_reps > 0:
        gl_h, genotype = genotype_leg(phmm, torch, ctx, batch, out, stream, args.genotype_reps)
        genotype["share_of_step"] = round(genotype["ms"] / ms_per_step, 5)
        if cpu is not None:
            genotype["parity_sample"] = genotype_parity(batch, args.cpu_regions, ovals, gl_h)
            log("genotype parity on %d sampled regions: ok=%s"
                % (genotype["parity_sample"]["regions"], genotype["parity_sample"]["ok"]))
        del gl_h

    end_to_end = None
    if args.end_to_end:
        # host arrays in, host results out (synchronous API): copies, device
        # packing, kernels and read-back; the first call sizes the arena
        with phmm.Context(timing=True) as hctx:
            if costs is not None:
                hctx.set_class_costs(costs)
            walls = []
            for r in range(2):
                t = time.perf_counter()
                phmm.phmm_forward_batch(hctx, batch)
                walls.append(time.perf_counter() - t)
                log("end-to-end call %d: %.2f s" % (r + 1, walls[-1]))
        end_to_end = dict(seconds=round(walls[-1], 3), gcups=round(cells / walls[-1] / 1e9, 1),
                          first_call_seconds=round(walls[0], 3),
                          note="host numpy arrays (pageable) in, host log10 L and flags out; "
                               "the second of two calls (the first also allocates the arena)")
    del db, ws
    torch.cuda.empty_cache()
    opw = one_pair_per_wave_leg(phmm, torch, args, costs) if args.opw_regions > 0 else None
    uneven = batched_uneven_leg(phmm, torch, args) if args.uneven else None
    small = small_batch_leg(phmm, torch, args) if args.small_reps > 0 else None
    long_reads = long_reads_leg(phmm, torch, args) if args.long_reps > 0 else None
    serving = serve_leg(phmm, args) if args.serve_seconds > 0 else None

    parity = None
    if cpu is not None:
        g = out_h[sidx]
        f = fl_h[sidx]
        fin = np.isfinite(ovals)
        d = np.where(fin, np.abs(np.where(fin, g, 0) - np.where(fin, ovals, 0)), 0.0)
        is32 = (f & phmm.PHMM_FLAG_FP32) != 0
        parity = dict(pairs=int(len(sidx)),
                      max_err_fp32=float(d[is32].max(initial=0.0)),
                      p99_err_fp32=float(np.percentile(d[is32], 99)) if is32.any() else 0.0,
                      max_err_fp64=float(d[~is32].max(initial=0.0)),
                      fp64_pairs=int((~is32).sum()),
                      ok=bool(d[is32].max(initial=0) <= 1e-4 and d[~is32].max(initial=0) <= 1e-10
                              and np.array_equal(np.isfinite(g), fin)))

    rec = dict(
        metric=METRIC, value=round(value, 2), unit="GCUPS", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(ms_per_step, 3),
        step_ms=dict(median=round(float(np.median(step_ms)), 3), min=round(min(step_ms), 3),
                     max=round(max(step_ms), 3), source="HIP events around each timed pass"),
        sclk_mhz=clock.summary(), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="genome-scale synthetic WGS-like batch: %d regions of 150 bp reads, "
                             "2-16 variant haplotypes of 150-600 bp, lognormal(mean 40, sigma 1) "
                             "reads per region, Phred 2-41; FP32 with FP64 rerun" % args.regions,
                    regions=args.regions, pairs=n_pairs, cells=cells),
        roofline=roof, cpu_baseline=cpu, cpu_rowform=rowform,
        phases_ms={k: round(v, 3) for k, v in ph.items()},
        rerun_pairs=int(counts["rerun_pairs"]), rerun_fraction=counts["rerun_pairs"] / max(1, n_pairs),
        lane_utilisation=round(cells32 / max(1, counts["lane_columns"] * 150), 4),
        pack_costs=None if costs is None else dict(fp32=np.round(costs[0], 3).tolist(),
                                                   fp64=np.round(costs[1], 3).tolist()),
        fp64_plain=fp64, fp64_one_pair_per_wave=opw, end_to_end=end_to_end,
        batched_uneven=uneven, small_batch=small, long_reads=long_reads, parity_sample=parity,
        serving=serving,
        genotype_likelihoods=genotype,
    )
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
