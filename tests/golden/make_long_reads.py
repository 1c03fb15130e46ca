"""Writes tests/golden/long_reads.json: oracle values of the longest reads.

The GPU parity tests compare the library with the oracle computed live, but
a read of 100,000 bases against a haplotype of 110,000 (the long-read
workload's longest class) and a read at the library's maximum length
(131,072 bases) take the single-threaded FP64 oracle about a minute each, so
their values are computed once here, by the oracle alone (rescaled form,
Section 2's model), from inputs the seeded generator recreates exactly.

Run:  python tests/golden/make_long_reads.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import synth  # noqa: E402

# (name, workload, first region): each region is one read x one haplotype
CASES = [
    ("long_read_100k", "long_reads", 64),
    ("max_read_131072", dict(synth.CONFIGS["long_reads"], regions=1, n_len_classes=1,
                             len_classes=(131072, 0, 0, 0), regions_per_class=1,
                             hap_len_factor=1.1), 0),
]


def main():
    out = {}
    for name, cfg, region in CASES:
        b = synth.generate(cfg, region, 1)
        t = time.time()
        v = float(oracle.forward_pairs(b, rescale=True)[0])
        out[name] = dict(region=region, read_len=int(b["read_offsets"][1]),
                         hap_len=int(b["hap_offsets"][1]), log10_l=repr(v))
        print(name, out[name], "%.1f s" % (time.time() - t), flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_reads.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
