"""The CPU comparator (row-level formulation with SIMD rows and threads over
pairs) against the oracle: FP32-accepted pairs within 1e-4 in log10, FP64
pairs within 1e-10, on variant and i.i.d. haplotypes, reads of 2048 bases
(every pair in FP64 with rescaling) and degenerate inputs."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import cpu_rowform  # noqa: E402
import oracle  # noqa: E402
import synth  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def built():
    cpu_rowform.build(force=False)


def check(batch, threads=4):
    got, flags = cpu_rowform.forward_pairs(batch, threads=threads)
    want = oracle.forward_pairs(batch)
    # a likelihood of exactly 0 (a base of Phred 0 against its own base) is
    # -inf on both sides
    fin = np.isfinite(want)
    np.testing.assert_array_equal(np.isfinite(got), fin)
    np.testing.assert_array_equal(got[~fin], want[~fin])
    d = np.where(fin, np.abs(np.where(fin, got, 0.0) - np.where(fin, want, 0.0)), 0.0)
    f32 = flags == 1
    assert set(np.unique(flags)) <= {1, 2}
    assert d[f32].max(initial=0) <= 1e-4, d[f32].max()
    assert d[~f32].max(initial=0) <= 1e-10, d[~f32].max()
    return flags


def test_variant_haplotypes():
    flags = check(synth.generate("batched_uneven", 0, 6))
    assert (flags == 1).mean() > 0.99


def test_iid_haplotypes_rerun_in_fp64():
    flags = check(synth.generate("one_region"))
    assert (flags == 2).any() and (flags == 1).any()


def test_long_pairs_rescaled():
    flags = check(synth.generate(synth.sweep_cfg(2048, 2), 0, 2), threads=8)
    assert np.all(flags == 2)


def test_degenerate_inputs_and_thread_counts():
    b = synth.generate("batched_uneven", 0, 1)
    one = dict(reads=np.frombuffer(b"ANGT", np.uint8), base_quals=np.array([0, 255, 30, 41], np.uint8),
               ins_quals=np.array([45, 0, 255, 45], np.uint8), del_quals=np.array([45, 255, 0, 45], np.uint8),
               gcp=np.array([10, 0, 255, 10], np.uint8), read_offsets=np.array([0, 1, 4], np.uint64),
               haplotypes=np.frombuffer(b"NACGTTGCA", np.uint8), hap_offsets=np.array([0, 1, 9], np.uint64),
               pair_list=np.array([[0, 0], [0, 1], [1, 0], [1, 1]], np.uint32))
    flags = check(one, threads=1)
    assert flags[1] == 1
    v1, _ = cpu_rowform.forward_pairs(b, threads=1)
    v8, _ = cpu_rowform.forward_pairs(b, threads=8)
    np.testing.assert_array_equal(v1, v8)
