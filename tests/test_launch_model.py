"""CPU checks of the launch protocol's control flow (tests/launch_model.py):
packer capacities and pack layout, the queues between kernel families and
the long kernel's ring pipeline, on the degenerate-input batch, on each of its
pairs alone and on synthetic batches, with the FP32/FP64 decisions taken from
the oracle and in the worst case (every pair rejected, every FP64 sum handed
to the long kernel)."""
import math

import numpy as np
import pytest

import oracle
import synth
from edge_batch import edge_pairs, make_batch
from launch_model import (LONG_TILE, RING, LaunchModel, ModelError, Policy, long_active_waves)

THRESH32 = -28.0 - 120 * math.log10(2.0)    # log10 L at an FP32 scaled sum of 1e-28
THRESH64 = -290.0 - 1020 * math.log10(2.0)  # FP64 scaled sums under 1e-290 go long


def single(b, q):
    """Pair q of a one-read-one-haplotype-per-pair batch, alone."""
    r, h = (int(x) for x in b["pair_list"][q])
    ro, ho = b["read_offsets"], b["hap_offsets"]
    out = dict(b)
    for key in ("reads", "base_quals", "ins_quals", "del_quals", "gcp"):
        out[key] = b[key][ro[r]:ro[r + 1]].copy()
    out["haplotypes"] = b["haplotypes"][ho[h]:ho[h + 1]].copy()
    out["read_offsets"] = np.array([0, ro[r + 1] - ro[r]], np.uint64)
    out["hap_offsets"] = np.array([0, ho[h + 1] - ho[h]], np.uint64)
    out["pair_list"] = np.array([[0, 0]], np.uint32)
    return out


def policies(b, **kw):
    n = len(b["pair_list"])
    kmax = int(np.diff(b["hap_offsets"].astype(np.int64)).max())
    for prec in (0, 1):
        yield Policy(precision=prec, **kw).for_batch(n, kmax)


def run_all_ways(b, grids=(None, None), **kw):
    want = oracle.forward_pairs(b, rescale=True)
    deciders = [
        (lambda q: want[q] >= THRESH32, lambda q: want[q] >= THRESH64),   # predicted path
        (lambda q: False, lambda q: False),                              # worst case
        (lambda q: True, lambda q: True),                                # nothing rejected
    ]
    for pol in policies(b, **kw):
        for acc32, ok64 in deciders:
            m = LaunchModel(b, pol)
            flags = m.run(acc32, ok64, grids)
            yield pol, m, flags


def test_edge_batch_protocol():
    """The batch of degenerate inputs (one-base reads and haplotypes, 'N',
    Phred 0 and 255, haplotypes of 256, 1536 and 1537 columns, per-row gap
    penalties): every queue stays within its capacity, every pair is written
    exactly once, and the long tiles complete, under both precisions and for
    any FP32/FP64 outcome."""
    b = make_batch(edge_pairs())
    n_runs = 0
    for pol, m, flags in run_all_ways(b):
        n_runs += 1
        assert pol.force_class == 20  # 1537 columns: the small batch's class holds 1536
        # the 1537-column pair is the only long pair from the packer
        long_from_packer = [q for q in range(m.n) if m.k_of(q) > 1536]
        assert long_from_packer == [9]
        # its read has one gap byte and insertion bytes of 45: the lean list
        assert 9 in m.long_list[0] or 9 in m.long_list[2]
    assert n_runs == 6


def test_edge_batch_l_zero_path():
    """Phred 0 everywhere gives T_DM = 0, so L = 0: the pair goes FP32 general
    kernel (gap byte 0) -> rejected -> FP64 item -> hand-off to the FP64 long
    kernel, where it is one tile."""
    b = make_batch(edge_pairs())
    want = oracle.forward_pairs(b, rescale=True)
    assert want[10] == -np.inf
    m = LaunchModel(b, Policy(precision=0).for_batch(len(b["pair_list"]), 1537))
    flags = m.run(lambda q: want[q] >= THRESH32, lambda q: want[q] >= THRESH64)
    assert 10 in m.long_list[3] and flags[10] == 0x1c
    assert flags[9] == 0x1c  # long pairs run in FP64 by default


@pytest.mark.parametrize("q", range(13))
def test_edge_pairs_alone(q):
    b = single(make_batch(edge_pairs()), q)
    for _ in run_all_ways(b):
        pass


@pytest.mark.parametrize("workload,seed,regions", [("batched_uneven", 1, 40),
                                                    ("genome_scale", 2, 20),
                                                    ("one_region", 0, None)])
def test_synthetic_batches_protocol(workload, seed, regions):
    b = synth.generate(workload, seed, regions) if regions else synth.generate(workload)
    for pol in policies(b):
        # full-size cost model choice (no small-batch forcing) and forced classes
        for fc in (-1, 0, 7, 20):
            p = Policy(precision=pol.precision, force_class=fc)
            m = LaunchModel(b, p)
            m.run(lambda q: True, lambda q: True)
            m = LaunchModel(b, p)
            m.run(lambda q: False, lambda q: False)


def long_batch(lengths, read_len, seed=3):
    rng = np.random.default_rng(seed)
    pairs = []
    for k in lengths:
        h = bytes(rng.choice(np.frombuffer(b"ACGT", np.uint8), k))
        pairs.append((h[:read_len], h, 30, 45, 45, 10))
    return make_batch(pairs)


def test_long_pair_beyond_stated_bound():
    """A long haplotype in a batch whose length bound says every haplotype
    fits the short kernels: no routing runs, the pair goes to the FP64
    general list (launched in every call) and the call reports the bound
    error; its output is still written once."""
    b = long_batch([100, 1600, 200], read_len=90)
    for prec in (0, 1):
        pol = Policy(precision=prec, long_fp32_max_rows=131072)
        m = LaunchModel(b, pol.for_batch(3, 1536))
        m.run(lambda q: True, lambda q: True)
        assert m.bound_error and m.long_list[3] == [1]
        assert not any(m.long_list[:3])
        m = LaunchModel(b, pol.for_batch(3, 1600))
        m.run(lambda q: True, lambda q: True)
        assert not m.bound_error and m.long_list[2 * prec] == [1]
    # by default long pairs run in FP64
    m = LaunchModel(b, Policy(precision=0).for_batch(3, 1600))
    m.run(lambda q: True, lambda q: True)
    assert m.long_list[2] == [1]


def test_long_pipeline_slot_reuse():
    """Many long pairs through few resident wavefronts: ring slots are taken
    over again and again (item it waits for item it - 2*grid), and the
    pipeline still drains."""
    b = long_batch([1537, 5000, 1024 * 7 + 3, 2048, 1600, 9000], read_len=700)
    for grid in (2, 3, 5, 64):
        m = LaunchModel(b, Policy(precision=1))
        m.run(lambda q: True, lambda q: True, grids=(grid, grid))


def test_long_grid_cut_to_tiles():
    """With fewer tiles than wavefronts only the first `tiles` wavefronts of
    the long kernel's grid take tiles (every tile still resident at once, so
    the pipeline drains); with more, every wavefront stays."""
    assert long_active_waves(1024, 4096) == 1024
    assert long_active_waves(6144, 4096) == 4096
    assert long_active_waves(0, 4096) == 4096
    b = long_batch([LONG_TILE * 40] * 3, read_len=RING * 3 + 5)  # 120 tiles on 300
    m = LaunchModel(b, Policy(precision=1))
    m.run(lambda q: True, lambda q: True, grids=(300, 300))


def test_long_pipeline_needs_resident_consumers():
    """A tile may run at most RING rows ahead of its consumer, and items are
    claimed in order, so a read longer than RING x (resident wavefronts) on a
    pair with more tiles than resident wavefronts cannot drain: the model
    reports the deadlock that the kernel's watchdog turns into PHMM_ETIMEOUT.
    The library launches a grid of every wavefront the chip holds (at least
    1024 for the FP64 kernel, more than the 1024 tiles of the longest
    haplotype), so its own launches stay clear of this."""
    tiles = 4
    b = long_batch([LONG_TILE * tiles], read_len=RING * 2 + 10)
    with pytest.raises(ModelError, match="deadlock"):
        LaunchModel(b, Policy(precision=1)).run(lambda q: True, lambda q: True, grids=(2, 2))
    LaunchModel(b, Policy(precision=1)).run(lambda q: True, lambda q: True, grids=(tiles, tiles))
