"""Writes tests/golden/long_reads_all.json: oracle values of all 96 pairs of
the long-read workload (32 reads each of 10,000, 32,000 and 100,000 bases
against haplotypes 1.1 times as long), for the benchmark's long-read leg and
the GPU tests.  The single-threaded FP64 oracle takes from under a second (10
kbp) to about a minute (100 kbp) per pair, so the values are computed once
here, by the oracle alone (rescaled form of Section 2's model), one pair per
worker process, from inputs the seeded generator recreates exactly.

Run:  python tests/golden/make_long_reads_all.py [workers]
"""
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import synth  # noqa: E402

N_PAIRS = 96


def one(region):
    b = synth.generate("long_reads", region, 1)
    t = time.time()
    v = float(oracle.forward_pairs(b, rescale=True)[0])
    return region, int(b["read_offsets"][1]), int(b["hap_offsets"][1]), v, time.time() - t


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    # longest pairs first, so the pool ends evenly
    order = sorted(range(N_PAIRS), key=lambda r: -r)
    out = {}
    with mp.Pool(workers) as pool:
        for region, l, k, v, sec in pool.imap_unordered(one, order):
            out[region] = dict(read_len=l, hap_len=k, log10_l=repr(v))
            print(region, l, k, v, "%.1f s" % sec, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_reads_all.json")
    with open(path, "w") as fh:
        json.dump({"workload": "long_reads", "pairs": [out[r] | {"region": r} for r in range(N_PAIRS)]},
                  fh, indent=0)
        fh.write("\n")


if __name__ == "__main__":
    main()
