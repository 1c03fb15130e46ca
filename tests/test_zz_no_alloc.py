"""phmm_forward_batch_noalloc (no workspace argument, no allocation: the
library's static device scratch) against phmm_forward_batch_async on the same
batches, through the C ABI: two calls in a row, the second on a smaller
batch, each bit-identical to the workspace call and within the oracle's
bounds on a sample."""
import ctypes
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import paper_2606_25738_amd as phmm  # noqa: E402
import synth  # noqa: E402
from edge_batch import make_batch, rnd  # noqa: E402

pytestmark = pytest.mark.gpu


def concat(a, b):
    """Two CSR batches as one (b's reads and haplotypes after a's)."""
    ra, ha = len(a["read_offsets"]) - 1, len(a["hap_offsets"]) - 1
    out = {}
    for k in ("reads", "base_quals", "ins_quals", "del_quals", "gcp", "haplotypes"):
        out[k] = np.concatenate([a[k], b[k]])
    out["read_offsets"] = np.concatenate([a["read_offsets"], a["read_offsets"][-1] + b["read_offsets"][1:]])
    out["hap_offsets"] = np.concatenate([a["hap_offsets"], a["hap_offsets"][-1] + b["hap_offsets"][1:]])
    pl = np.asarray(b["pair_list"], np.uint32).copy()
    pl[:, 0] += ra
    pl[:, 1] += ha
    out["pair_list"] = np.concatenate([np.asarray(a["pair_list"], np.uint32), pl])
    return out


def long_pairs(seed):
    rng = np.random.default_rng(seed)
    pairs = []
    for k, l in ((3000, 600), (5200, 2000), (1700, 1500)):
        hap = rnd(rng, k)
        off = int(rng.integers(0, k - l))
        rd = bytearray(hap[off:off + l])
        for p in rng.choice(l, l // 50, replace=False):
            rd[p] = ord("ACGT"[int(rng.integers(0, 4))])
        pairs.append((bytes(rd), hap, rng.integers(10, 41, l), 40, 40, 10))
    return make_batch(pairs)


def run(ctx, b, noalloc):
    import torch
    db = phmm.DeviceBatch(b)
    n = db.n_pairs
    out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
    fl = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.Stream()
    if noalloc:
        phmm.phmm_forward_batch_noalloc(ctx, db, out, fl, s)
    else:
        ws = torch.empty(phmm.phmm_workspace_bytes(ctx, n, db.max_read_len, db.max_hap_len),
                         dtype=torch.uint8, device="cuda:0")
        phmm.phmm_forward_batch_async(ctx, db, out, fl, ws, s)
    s.synchronize()
    return out.cpu().numpy(), fl.cpu().numpy()


def test_noalloc_matches_workspace_call():
    big = concat(synth.generate("batched_uneven", 2, 50), long_pairs(1))
    small = concat(synth.generate("batched_uneven", 9, 4), long_pairs(2))
    assert len(big["pair_list"]) > 8192 > len(small["pair_list"])
    with phmm.Context() as c:
        for name, b in (("big", big), ("small", small)):
            print("noalloc call on %s batch: %d pairs" % (name, len(b["pair_list"])), flush=True)
            got, gf = run(c, b, True)
            want, wf = run(c, b, False)
            assert np.array_equal(gf, wf)
            assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
            n = len(got)
            idx = np.concatenate([np.arange(0, n - 3, max(1, n // 150)), np.arange(n - 3, n)])
            ref = oracle.forward_pairs(b, idx, rescale=True)
            is32 = (gf[idx] & phmm.PHMM_FLAG_FP32) != 0
            d = np.abs(got[idx] - ref)
            assert d[is32].max(initial=0) <= 1e-4 and d[~is32].max(initial=0) <= 1e-10
            assert np.all(gf[-3:] & phmm.PHMM_FLAG_LONG)


def test_noalloc_rejects_batches_over_its_limit():
    """A batch beyond PHMM_NOALLOC_MAX_PAIRS is refused before any device
    work (the pointers are never read)."""
    from paper_2606_25738_amd._binding import _DeviceBatch
    s = _DeviceBatch()
    s.n_pairs = (1 << 19) + 1
    with phmm.Context() as c:
        rc = phmm.lib().phmm_forward_batch_noalloc(c.handle, ctypes.byref(s), None, None, None)
    assert rc == phmm.PHMM_ERANGE
    assert b"exceed" in phmm.lib().phmm_last_error()
