"""The serving runtime (phmm_server_*) on the GPU: results of regions served
in a mix equal those of each region alone, long regions take the long lane,
polling, admission limits, CU-masked lanes."""
import os
import sys
import threading
import time

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import paper_2606_25738_amd as phmm  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

TOL32 = 1e-4
TOL64 = 1e-10
THRESH = -64.1236


def say(*a):
    print(*a, flush=True)


LONG_READ_MIN = 512  # the server's default routing bound


@pytest.fixture(scope="module")
def stream_regions():
    """A mixed stream: 160 regions of the served workload (short regions and
    long-read regions), cut short so the test stays quick."""
    b = synth.generate("served_stream", 0, 160)
    regs = [synth.region_slice(b, i) for i in range(160)]
    nlong = sum(int(np.diff(r["read_offsets"]).max() > LONG_READ_MIN or
                    np.diff(r["hap_offsets"]).max() > 1536) for r in regs)
    say("served stream sample: %d regions, %d long, %.3g cells" %
        (len(regs), nlong, sum(synth.batch_cells(r) for r in regs)))
    return regs


def compare(a, fa, b, fb, near=None):
    """Same results up to the rounding of a different wavefront position."""
    fin = np.isfinite(a)
    assert np.array_equal(fin, np.isfinite(b))
    d = np.abs(np.where(fin, a, 0) - np.where(fin, b, 0))
    same = fa == fb
    if near is not None:  # a pair on the acceptance threshold may land either side
        same |= np.abs(a - THRESH) < 1e-3
    assert same.all(), "flags differ"
    is32 = (fa & phmm.PHMM_FLAG_FP32) != 0
    assert d[is32].max(initial=0) <= 1e-5
    assert d[~is32].max(initial=0) <= 1e-12


def test_mix_equals_alone(stream_regions):
    regs = stream_regions
    with phmm.Context() as ctx:
        alone = [phmm.phmm_forward_batch(ctx, r) for r in regs]
    with phmm.Server(lanes=3, long_lanes=1, hbm_budget_bytes=6 << 30) as srv:
        tickets = [None] * len(regs)

        def submitter(idx):
            rng = np.random.default_rng(idx[0])
            for i in idx:
                tickets[i] = srv.submit(regs[i])
                time.sleep(float(rng.exponential(0.0005)))
        th = [threading.Thread(target=submitter, args=(list(range(k, len(regs), 2)),))
              for k in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    say("server: %d batches for %d regions, busy %.3f s" % (st["batches"], st["regions"],
                                                         st["lane_busy_s"]))
    assert st["regions"] == len(regs) and st["batches"] >= 2
    for (a, fa), (b, fb, info) in zip(alone, got):
        compare(a, fa, b, fb, near=True)
        assert info["n_pairs"] == len(a) and info["latency_s"] >= info["queue_s"] >= 0
    # the long lane took every long region (a read over 512 bases or a
    # haplotype over 64 x 24 columns, the server's defaults)
    for r, (_, _, info) in zip(regs, got):
        is_long = (np.diff(r["read_offsets"]).max() > LONG_READ_MIN or
                   np.diff(r["hap_offsets"]).max() > 1536)
        assert info["is_long"] == int(is_long)
        if is_long:
            assert info["lane"] == 2
        else:
            assert info["lane"] in (0, 1)


def test_served_short_regions_match_oracle(stream_regions):
    short = [r for r in stream_regions
             if np.diff(r["hap_offsets"]).max() <= 1536 and np.diff(r["read_offsets"]).max() <= 2048]
    rng = np.random.default_rng(4)
    pick = [short[i] for i in rng.choice(len(short), size=min(12, len(short)), replace=False)]
    with phmm.Server(lanes=2, long_lanes=0, hbm_budget_bytes=2 << 30) as srv:
        ts = [srv.submit(r) for r in pick]
        res = [srv.wait(t) for t in ts]
    for r, (out, fl, _) in zip(pick, res):
        want = oracle.forward_pairs(r, np.arange(len(out)), rescale=True)
        fin = np.isfinite(want)
        d = np.abs(np.where(fin, out, 0) - np.where(fin, want, 0))
        is32 = (fl & phmm.PHMM_FLAG_FP32) != 0
        assert d[is32].max(initial=0) <= TOL32 and d[~is32].max(initial=0) <= TOL64


def test_served_long_regions_match_oracle(stream_regions):
    """Long-read regions through the long lane (capped grids), with short
    regions running beside them: sampled pairs of the shortest long regions
    against the oracle."""
    longs = [r for r in stream_regions if np.diff(r["read_offsets"]).max() > LONG_READ_MIN]
    longs.sort(key=lambda r: int(np.diff(r["read_offsets"]).max()))
    pick = longs[:3]
    short = [r for r in stream_regions if np.diff(r["read_offsets"]).max() <= LONG_READ_MIN][:40]
    assert pick and short
    # long lanes on half the chip's persistent grid
    with phmm.Server(lanes=3, long_lanes=1, hbm_budget_bytes=6 << 30,
                     long_grid_percent=50) as srv:
        ts = [srv.submit(r) for r in pick + short]
        res = [srv.wait(t) for t in ts]
    rng = np.random.default_rng(9)
    for r, (out, fl, info) in zip(pick, res):
        assert info["is_long"] == 1 and info["lane"] == 2
        idx = np.sort(rng.choice(len(out), size=min(3, len(out)), replace=False))
        say("served long region: read %d bases, %d pairs, checking %s" %
            (int(np.diff(r["read_offsets"]).max()), len(out), idx.tolist()))
        want = oracle.forward_pairs(r, idx, rescale=True)
        d = np.abs(out[idx] - want)
        is32 = (fl[idx] & phmm.PHMM_FLAG_FP32) != 0
        assert d[is32].max(initial=0) <= TOL32 and d[~is32].max(initial=0) <= TOL64


def test_poll_and_budget_limit():
    b = synth.generate("genome_scale", 0, 3)
    r = synth.region_slice(b, 0)
    with phmm.Server(lanes=2, long_lanes=0, hbm_budget_bytes=512 << 20) as srv:
        t = srv.submit(r)
        res = None
        for _ in range(20000):
            res = srv.poll(t)
            if res is not None:
                break
            time.sleep(0.0005)
        assert res is not None
        with phmm.Context() as ctx:
            a, fa = phmm.phmm_forward_batch(ctx, r)
        compare(a, fa, res[0], res[1])
        # a region larger than one lane's share (256 MiB) is refused at once:
        # 8M pairs need about 45 bytes each of pair list, outputs and workspace
        n_haps, n_pairs = 3000, 8_000_000
        huge = {k: r[k][:100] for k in ("reads", "base_quals", "ins_quals", "del_quals", "gcp")}
        huge["read_offsets"] = np.array([0, 100], np.uint64)
        huge["haplotypes"] = np.tile(np.frombuffer(b"ACGTACGTAC", np.uint8), n_haps)
        huge["hap_offsets"] = np.arange(n_haps + 1, dtype=np.uint64) * 10
        huge["pair_list"] = np.stack([np.zeros(n_pairs), np.arange(n_pairs) % n_haps],
                                     1).astype(np.uint32)
        with pytest.raises(phmm.PhmmError) as e:
            srv.submit(huge)
        assert e.value.code == phmm.PHMM_ENOMEM


def test_cu_masked_lanes(stream_regions):
    regs = stream_regions[:60]
    with phmm.Server(lanes=3, long_lanes=1, short_cu_percent=25, hbm_budget_bytes=6 << 30) as srv:
        ts = [srv.submit(r) for r in regs]
        got = [srv.wait(t) for t in ts]
        st = srv.stats()
    say("cu mask status %d" % st["cu_mask_status"])
    assert st["cu_mask_status"] != 0
    with phmm.Context() as ctx:
        for r, (b, fb, _) in zip(regs, got):
            a, fa = phmm.phmm_forward_batch(ctx, r)
            compare(a, fa, b, fb, near=True)


def test_lanes_have_their_own_queues(stream_regions):
    """With default options every lane's stream is CU-masked (all compute
    units), which gives it a hardware queue of its own: streams the process
    created before the server cannot put a short lane behind a long one."""
    import torch
    others = [torch.cuda.Stream() for _ in range(4)]
    for s in others:
        with torch.cuda.stream(s):
            torch.ones(16, device="cuda:0").sum()
    torch.cuda.synchronize()
    regs = stream_regions[:20]
    with phmm.Server(hbm_budget_bytes=3 << 30) as srv:
        ts = [srv.submit(r) for r in regs]
        got = [srv.wait(t) for t in ts]
        st = srv.stats()
    assert st["cu_mask_status"] == 1
    with phmm.Context() as ctx:
        for r, (b, fb, _) in zip(regs, got):
            a, fa = phmm.phmm_forward_batch(ctx, r)
            compare(a, fa, b, fb, near=True)


def test_budget_admission_splits_batches():
    """Regions submitted faster than they run wait in the queue; a lane takes
    them in order while its batch still fits its share of the HBM budget.
    3200 regions of one 10 kbp read against one 11 kbp haplotype (the
    long-read workload's shortest class, each submitted 100 times; about
    60 KB each, 1.1e8 cells) go to one lane of 168 MiB, of which the long
    kernels' rings take 128 MiB: they go out in several batches, some cut
    short by the budget (the server's full-batch count), and every region's
    results equal those of the region run alone."""
    b = synth.generate("long_reads")
    uniq = [synth.region_slice(b, i) for i in range(32)]
    assert all(int(np.diff(r["read_offsets"]).max()) == 10000 for r in uniq)
    with phmm.Context() as ctx:
        alone = [phmm.phmm_forward_batch(ctx, r) for r in uniq]
    with phmm.Server(lanes=1, long_lanes=0, hbm_budget_bytes=168 << 20) as srv:
        st0 = srv.stats()
        ts = [srv.submit(uniq[i % 32]) for i in range(3200)]
        got = [srv.wait(t) for t in ts]
        st = srv.stats()
    nb = st["batches"] - st0["batches"]
    nfull = st["full_batches"] - st0["full_batches"]
    say("budget admission: 3200 regions in %d batches, %d cut short by the budget" % (nb, nfull))
    assert nfull >= 1 and nb >= 3
    for i, (o, fo, _) in enumerate(got):
        a, fa = alone[i % 32]
        compare(a, fa, o, fo)
