"""Seeded synthetic PairHMM workloads shaped like the paper's inputs.

Only sequences and quality bytes are drawn here; no PairHMM arithmetic.
Both the tests (oracle side) and the benchmark (product side) use this
module, so the same seed always produces the same batch.

A batch is a dict of numpy arrays in the CSR layout of the library's
boundary:

  reads, base_quals, ins_quals, del_quals, gcp : uint8, concatenated reads
  read_offsets                                 : uint64, n_reads + 1
  haplotypes                                   : uint8, concatenated
  hap_offsets                                  : uint64, n_haps + 1
  pair_list                                    : uint32, (n_pairs, 2) = (read, hap)
  region_pairs                                 : uint64, first pair of each region (+ end)
  cols (optional)                              : int32, per read base the aligned
                                                 1-based hap column (0 = inserted
                                                 base, -1 = overhang / no true path)

Workloads (the paper's real data sets are not available; these stand in for
them with the published shapes only):

  one_region      one region, 8 i.i.d. haplotypes x 200 bp, 64 reads x 100 bp
  batched_uneven  20,000 regions, 2-8 variant haplotypes of 150-600 bp,
                  lognormal reads (mean 40, sigma 1, cap 400) of 100-150 bp
  long_reads      96 long pairs: 32 each of 10k, 32k and 100k bp, haplotype
                  1.1x read
  genome_scale    regions of 150 bp reads, 2-16 variant haplotypes of
                  150-600 bp, lognormal read counts, qualities Phred 2-41
  served_stream   genome_scale regions, 5% of them long-read regions (reads
                  of 1k-20k bp, 2-4 haplotypes of 1.1x read length)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "libsynth.so")


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("n_haps_lo", ctypes.c_int), ("n_haps_hi", ctypes.c_int),
        ("hap_len_lo", ctypes.c_int), ("hap_len_hi", ctypes.c_int),
        ("hap_mode", ctypes.c_int),
        ("var_lo", ctypes.c_int), ("var_hi", ctypes.c_int),
        ("var_snp_frac", ctypes.c_double),
        ("var_indel_lo", ctypes.c_int), ("var_indel_hi", ctypes.c_int),
        ("reads_mode", ctypes.c_int), ("reads_fixed", ctypes.c_int),
        ("reads_mu", ctypes.c_double), ("reads_sigma", ctypes.c_double),
        ("reads_cap", ctypes.c_int),
        ("read_len_lo", ctypes.c_int), ("read_len_hi", ctypes.c_int),
        ("n_len_classes", ctypes.c_int), ("len_classes", ctypes.c_int * 4),
        ("regions_per_class", ctypes.c_int),
        ("hap_len_factor", ctypes.c_double),
        ("p_sub", ctypes.c_double), ("p_indel", ctypes.c_double),
        ("indel_lo", ctypes.c_int), ("indel_hi", ctypes.c_int),
        ("q_lo", ctypes.c_int), ("q_hi", ctypes.c_int),
        ("ins_q", ctypes.c_int), ("del_q", ctypes.c_int), ("gcp_q", ctypes.c_int),
        ("offset_mode", ctypes.c_int), ("offset_frac", ctypes.c_double),
        ("long_frac", ctypes.c_double), ("long_len_lo", ctypes.c_int),
        ("long_len_hi", ctypes.c_int), ("long_haps_lo", ctypes.c_int),
        ("long_haps_hi", ctypes.c_int), ("long_hap_factor", ctypes.c_double),
    ]


class _Sizes(ctypes.Structure):
    _fields_ = [("n_haps", ctypes.c_uint64), ("hap_bases", ctypes.c_uint64),
                ("n_reads", ctypes.c_uint64), ("read_bases", ctypes.c_uint64),
                ("n_pairs", ctypes.c_uint64)]


_LOGN_MU = math.log(40.0) - 0.5  # lognormal with mean 40 and sigma 1

_BASE = dict(n_haps_lo=8, n_haps_hi=8, hap_len_lo=200, hap_len_hi=200, hap_mode=0,
             var_lo=1, var_hi=3, var_snp_frac=0.8, var_indel_lo=1, var_indel_hi=5,
             reads_mode=0, reads_fixed=64, reads_mu=_LOGN_MU, reads_sigma=1.0,
             reads_cap=400, read_len_lo=100, read_len_hi=100, n_len_classes=0,
             len_classes=(0, 0, 0, 0), regions_per_class=1, hap_len_factor=0.0,
             p_sub=0.01, p_indel=0.001, indel_lo=1, indel_hi=3, q_lo=10, q_hi=40,
             ins_q=45, del_q=45, gcp_q=10, offset_mode=0, offset_frac=0.0,
             long_frac=0.0, long_len_lo=0, long_len_hi=0, long_haps_lo=0, long_haps_hi=0,
             long_hap_factor=0.0)

CONFIGS = {
    # one region, plain FP64 (8 i.i.d. haps x 200 bp, 64 reads x 100 bp)
    "one_region": dict(_BASE, regions=1, seed=0),
    # batched uneven short pairs
    "batched_uneven": dict(_BASE, regions=20000, seed=1, n_haps_lo=2, n_haps_hi=8, hap_len_lo=150,
                 hap_len_hi=600, hap_mode=1, reads_mode=1, read_len_lo=100, read_len_hi=150),
    # long-read pairs (one read x one hap per region), 32 each of three lengths
    "long_reads": dict(_BASE, regions=96, seed=2, n_haps_lo=1, n_haps_hi=1, reads_fixed=1,
                 n_len_classes=3, len_classes=(10000, 32000, 100000, 0), regions_per_class=32,
                 hap_len_factor=1.1, p_sub=0.05, p_indel=0.02, indel_lo=1, indel_hi=10,
                 q_lo=5, q_hi=30, ins_q=30, del_q=30, offset_mode=1, offset_frac=0.05),
    # genome-scale WGS-like regions (generated in chunks of regions)
    "genome_scale": dict(_BASE, regions=1000000, seed=3, n_haps_lo=2, n_haps_hi=16, hap_len_lo=150,
                 hap_len_hi=600, hap_mode=1, reads_mode=1, read_len_lo=150, read_len_hi=150,
                 p_sub=0.005, p_indel=0.0005, q_lo=2, q_hi=41),
}
# served request stream: regions as in the genome-scale workload, 5% of them
# long (all reads of one length U{1000..20000}, 2-4 haplotypes of 1.1x that
# length, same error and quality model); the region count is a pool the
# arrival process draws from in order
CONFIGS["served_stream"] = dict(CONFIGS["genome_scale"], regions=1000000, seed=4, long_frac=0.05,
                       long_len_lo=1000, long_len_hi=20000, long_haps_lo=2, long_haps_hi=4,
                       long_hap_factor=1.1)

_lock = threading.Lock()
_lib = None


def iid_haps_cfg(name: str = "batched_uneven") -> dict:
    """The stress variant of a workload: the same recipe with every haplotype
    drawn i.i.d. instead of as variants of one source haplotype, so that a
    read matches one haplotype of its region and most of its pairs fall far
    below FP32's range (and rerun in FP64)."""
    return dict(CONFIGS[name], hap_mode=0)


def small_batch_cfg() -> dict:
    """A small latency batch shaped like the paper's short-read test set (about
    3550 pairs of reads and haplotypes up to 263 bases): 71 regions of 10
    reads (100-150 bp) against 5 variant haplotypes of 150-263 bp; error and
    quality model as in the one-region workload."""
    return dict(_BASE, regions=71, seed=6, n_haps_lo=5, n_haps_hi=5, hap_len_lo=150,
                hap_len_hi=263, hap_mode=1, reads_mode=0, reads_fixed=10, read_len_lo=100,
                read_len_hi=150)


def sweep_cfg(length: int, regions: int) -> dict:
    """Equal-length pairs for the length sweep: per region one read of
    `length` bases against 16 haplotypes of `length` bases (variants of one
    source haplotype by 1-3 SNPs, so all keep the length); 1% substitutions,
    0.1% indels of 1-3 bp in the read; base quality U{10..40}, ins/del 45,
    gcp 10."""
    return dict(_BASE, regions=regions, seed=5, n_haps_lo=16, n_haps_hi=16,
                hap_len_lo=length, hap_len_hi=length, hap_mode=1, var_snp_frac=1.0,
                reads_mode=0, reads_fixed=1, read_len_lo=length, read_len_hi=length)



def build_synth(force: bool = True) -> str:
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-std=c11", "-fPIC", "-shared", _SRC,
                        "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build_synth(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.POINTER
            u64p, u8p = P(ctypes.c_uint64), P(ctypes.c_uint8)
            lib.synth_size.argtypes = [P(_Cfg), ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_uint64, P(_Sizes)]
            lib.synth_fill.argtypes = [P(_Cfg), ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       u64p, u64p, u64p, u64p, u64p,
                                       u8p, u64p, u8p, u8p, u8p, u8p, u8p, u64p,
                                       P(ctypes.c_uint32), P(ctypes.c_int32)]
            lib.synth_size.restype = ctypes.c_int
            lib.synth_fill.restype = ctypes.c_int
            _lib = lib
    return _lib


def make_cfg(name_or_dict, **overrides) -> dict:
    d = dict(CONFIGS[name_or_dict]) if isinstance(name_or_dict, str) else dict(name_or_dict)
    d.update(overrides)
    return d


def _to_struct(d: dict) -> _Cfg:
    c = _Cfg()
    for name, _ in _Cfg._fields_:
        v = d[name]
        if name == "len_classes":
            arr = (ctypes.c_int * 4)(*list(v))
            c.len_classes = arr
        else:
            setattr(c, name, v)
    return c


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def generate(cfg, region_start: int = 0, region_count: int | None = None,
             seed: int | None = None, with_cols: bool = False) -> dict:
    """Generate regions [region_start, region_start + region_count) of a
    workload.  ``cfg`` is a config name or dict; the default seed is the
    workload's own."""
    d = make_cfg(cfg) if isinstance(cfg, str) else dict(cfg)
    if seed is None:
        seed = d.get("seed", 0)
    if region_count is None:
        region_count = d["regions"] - region_start
    lib = _load()
    c = _to_struct(d)
    n = int(region_count)
    sizes = (_Sizes * n)()
    if lib.synth_size(ctypes.byref(c), seed, region_start, n, sizes) != 0:
        raise MemoryError("synth_size failed")
    sz = np.ctypeslib.as_array(sizes).view(np.uint64).reshape(n, 5)
    cnt = {k: sz[:, i].astype(np.uint64) for i, k in
           enumerate(("n_haps", "hap_bases", "n_reads", "read_bases", "n_pairs"))}
    pref = {k: np.concatenate([[0], np.cumsum(v)]).astype(np.uint64) for k, v in cnt.items()}
    tot = {k: int(v[-1]) for k, v in pref.items()}
    haps = np.empty(tot["hap_bases"], np.uint8)
    hap_off = np.empty(tot["n_haps"] + 1, np.uint64)
    rb = tot["read_bases"]
    reads, bq, iq, dq, gq = (np.empty(rb, np.uint8) for _ in range(5))
    read_off = np.empty(tot["n_reads"] + 1, np.uint64)
    pairs = np.empty((tot["n_pairs"], 2), np.uint32)
    cols = np.empty(rb, np.int32) if with_cols else None
    u64 = ctypes.c_uint64
    rc = lib.synth_fill(ctypes.byref(c), seed, region_start, n,
                        _ptr(pref["n_haps"], u64), _ptr(pref["hap_bases"], u64),
                        _ptr(pref["n_reads"], u64), _ptr(pref["read_bases"], u64),
                        _ptr(pref["n_pairs"], u64),
                        _ptr(haps, ctypes.c_uint8), _ptr(hap_off, u64),
                        _ptr(reads, ctypes.c_uint8), _ptr(bq, ctypes.c_uint8),
                        _ptr(iq, ctypes.c_uint8), _ptr(dq, ctypes.c_uint8),
                        _ptr(gq, ctypes.c_uint8), _ptr(read_off, u64),
                        _ptr(pairs, ctypes.c_uint32),
                        _ptr(cols, ctypes.c_int32) if with_cols else None)
    if rc != 0:
        raise MemoryError("synth_fill failed")
    hap_off[-1] = tot["hap_bases"]
    read_off[-1] = tot["read_bases"]
    out = dict(reads=reads, base_quals=bq, ins_quals=iq, del_quals=dq, gcp=gq,
               read_offsets=read_off, haplotypes=haps, hap_offsets=hap_off,
               pair_list=pairs, region_pairs=pref["n_pairs"],
               region_reads=pref["n_reads"], region_haps=pref["n_haps"])
    if with_cols:
        out["cols"] = cols
    return out


def batch_cells(batch: dict) -> int:
    """Number of DP cells sum(l * k) over the batch's pairs."""
    rl = np.diff(batch["read_offsets"]).astype(np.int64)
    hl = np.diff(batch["hap_offsets"]).astype(np.int64)
    pl = batch["pair_list"]
    return int(np.sum(rl[pl[:, 0]] * hl[pl[:, 1]]))


def subset_pairs(batch: dict, pair_idx) -> dict:
    """Same inputs, restricted pair list."""
    out = dict(batch)
    out["pair_list"] = np.ascontiguousarray(batch["pair_list"][np.asarray(pair_idx)])
    return out


def region_slice(batch: dict, i: int) -> dict:
    """Region i of a generated batch as a batch of its own (local offsets)."""
    rp, rr, rh = batch["region_pairs"], batch["region_reads"], batch["region_haps"]
    r0, r1 = int(rr[i]), int(rr[i + 1])
    h0, h1 = int(rh[i]), int(rh[i + 1])
    ro = batch["read_offsets"][r0:r1 + 1]
    ho = batch["hap_offsets"][h0:h1 + 1]
    b0, b1 = int(ro[0]), int(ro[-1])
    out = {k: batch[k][b0:b1] for k in ("reads", "base_quals", "ins_quals", "del_quals", "gcp")}
    out["read_offsets"] = (ro - ro[0]).astype(np.uint64)
    out["haplotypes"] = batch["haplotypes"][int(ho[0]):int(ho[-1])]
    out["hap_offsets"] = (ho - ho[0]).astype(np.uint64)
    pl = batch["pair_list"][int(rp[i]):int(rp[i + 1])].astype(np.int64)
    out["pair_list"] = np.stack([pl[:, 0] - r0, pl[:, 1] - h0], axis=1).astype(np.uint32)
    return out


def genotype_lk(seed: int, n_regions: int, reads=(0, 60), haps=(1, 16), long_frac: float = 0.0):
    """Synthetic read x haplotype log10-likelihood matrices shaped like the
    PairHMM output of active regions (the input of the genotyping step).

    Per region: R reads (uniform in [reads[0], reads[1]]) and H haplotypes
    (uniform in [haps[0], haps[1]]).  Per read, one haplotype it was drawn
    from scores -U(1, 25) (150 bp reads with sequencing errors); the others
    trail it by Exp(mean 8) (a few mismatching bases), 10% of them by
    U(50, 400) (an unrelated haplotype).  A long_frac share of the regions
    has long-read values (-U(1e3, 3e4) for the best haplotype).

    Returns (lk float64, lk_offsets uint64, region_reads uint32, region_haps
    uint32) with the regions' R x H blocks back to back, read-major."""
    g = np.random.default_rng(np.random.PCG64(seed))
    R = g.integers(reads[0], reads[1] + 1, n_regions).astype(np.uint32)
    H = g.integers(haps[0], haps[1] + 1, n_regions).astype(np.uint32)
    sizes = R.astype(np.int64) * H.astype(np.int64)
    off = np.zeros(n_regions, np.uint64)
    if n_regions > 1:
        off[1:] = np.cumsum(sizes[:-1]).astype(np.uint64)
    n = int(sizes.sum())
    lk = np.empty(n, np.float64)
    longr = g.random(n_regions) < long_frac
    for i in range(n_regions):
        r, h = int(R[i]), int(H[i])
        if r == 0:
            continue
        top = -(g.uniform(1e3, 3e4, r) if longr[i] else g.uniform(1.0, 25.0, r))
        gap = g.exponential(8.0, (r, h))
        far = g.random((r, h)) < 0.1
        gap[far] = g.uniform(50.0, 400.0, int(far.sum()))
        gap[np.arange(r), g.integers(0, h, r)] = 0.0
        o = int(off[i])
        lk[o:o + r * h] = (top[:, None] - gap).ravel()
    return lk, off, R, H
