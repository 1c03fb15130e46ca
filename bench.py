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
import json
import math
import multiprocessing as mp
import os
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


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _oracle_chunk(idx):
    import oracle
    t = time.process_time()
    v = oracle.forward_pairs(_BATCH, idx, rescale=True)
    return v, time.process_time() - t


def sample_pairs(batch, n_regions, seed=123):
    rp = batch["region_pairs"]
    nreg = len(rp) - 1
    rng = np.random.default_rng(seed)
    regs = np.sort(rng.choice(nreg, size=min(n_regions, nreg), replace=False))
    return np.concatenate([np.arange(rp[r], rp[r + 1]) for r in regs]).astype(np.int64), len(regs)


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


def pair_cells(batch):
    rl = np.diff(batch["read_offsets"]).astype(np.int64)
    hl = np.diff(batch["hap_offsets"]).astype(np.int64)
    pl = batch["pair_list"]
    return rl[pl[:, 0]] * hl[pl[:, 1]], rl[pl[:, 0]], hl[pl[:, 1]]


def time_steps(phmm, torch, ctx, db, out, fl, ws, stream, warmup, steps):
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
    return elapsed, avg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--regions", type=int, default=1000000,
                    help="regions of the workload (default: all 1,000,000)")
    ap.add_argument("--cpu-regions", type=int, default=1500,
                    help="regions in the oracle sample (CPU baseline and sampled parity)")
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="timed steps of the plain FP64 path on the same batch (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    t = time.perf_counter()
    batch = synth.generate("cfg3", 0, args.regions)
    cells_pp, rl, hl = pair_cells(batch)
    cells = int(cells_pp.sum())
    n_pairs = len(cells_pp)
    log("generated %d regions, %d pairs, %.4g cells in %.1fs"
        % (args.regions, n_pairs, cells, time.perf_counter() - t))

    # oracle sample first: worker processes fork before the GPU is touched
    cores = min(16, os.cpu_count() or 1)
    cpu = None
    if not args.no_cpu and args.cpu_regions > 0:
        sidx, nreg = sample_pairs(batch, args.cpu_regions)
        scells = int(cells_pp[sidx].sum())
        log("oracle on %d pairs (%d regions, %.3g cells), %d processes" % (len(sidx), nreg, scells, cores))
        ovals, wall, cpusec = run_oracle(batch, sidx, cores)
        cpu = dict(value=round(scells / wall / 1e9, 4), unit="GCUPS", cores=cores, kind="oracle",
                   sample="%d random regions of the same workload (%d pairs, %.3g cells); "
                          "single-core %.3f GCUPS" % (nreg, len(sidx), scells,
                                                       scells / cpusec / 1e9),
                   seconds=round(wall, 2))
        log("oracle %.1fs wall, %.3f GCUPS on %d processes" % (wall, cpu["value"], cores))

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
    ws = torch.empty(phmm.phmm_workspace_bytes(ctx, n_pairs, db.max_read_len, db.max_hap_len),
                     dtype=torch.uint8, device="cuda:0")
    elapsed, ph = time_steps(phmm, torch, ctx, db, out, fl, ws, stream, args.warmup, args.steps)
    counts = phmm.phmm_last_counts(ctx, ws)
    ms_per_step = elapsed * 1000.0 / args.steps
    value = cells / (elapsed / args.steps) / 1e9
    out_h = out.cpu().numpy()
    fl_h = fl.cpu().numpy()

    # dominant kernel: the FP32 short-pair kernels (one launch per column class)
    short = (hl <= 64 * 24)
    cells32 = int(cells_pp[short].sum())
    achieved = FLOPS_PER_CELL * cells32 / (ph["short_ms"] / 1e3) / 1e12
    roof = dict(bound="alu", achieved=round(achieved, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                frac=round(achieved / FP32_PEAK_TFLOPS, 4), traffic=None,
                kernel="FP32 short-pair kernels (11 column-class launches per step)",
                kernel_ms=round(ph["short_ms"], 3),
                measured_peak_fp32=round(peak32, 2), measured_peak_fp64=round(peak64, 2),
                frac_of_measured=round(achieved / peak32, 4))

    fp64 = None
    if args.fp64_steps > 0:
        ctx64 = phmm.Context(precision=phmm.PHMM_FP64_PLAIN, timing=True)
        out64 = torch.empty_like(out)
        fl64 = torch.empty_like(fl)
        e64, ph64 = time_steps(phmm, torch, ctx64, db, out64, fl64, ws, stream, 1, args.fp64_steps)
        fp64 = dict(gcups=round(cells / (e64 / args.fp64_steps) / 1e9, 2),
                    ms_per_step=round(e64 * 1000 / args.fp64_steps, 2),
                    speedup_fp32_rerun=round(value / (cells / (e64 / args.fp64_steps) / 1e9), 3))
        ctx64.close()

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
        warmup=args.warmup, ms_per_step=round(ms_per_step, 3), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="genome-scale synthetic WGS-like batch: %d regions of 150 bp reads, "
                             "2-16 variant haplotypes of 150-600 bp, lognormal(mean 40, sigma 1) "
                             "reads per region, Phred 2-41; FP32 with FP64 rerun" % args.regions,
                    regions=args.regions, pairs=n_pairs, cells=cells),
        roofline=roof, cpu_baseline=cpu,
        phases_ms={k: round(v, 3) for k, v in ph.items()},
        rerun_pairs=int(counts["rerun_pairs"]), rerun_fraction=counts["rerun_pairs"] / max(1, n_pairs),
        lane_utilisation=round(cells32 / max(1, counts["lane_columns"] * 150), 4),
        fp64_plain=fp64, parity_sample=parity,
    )
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
