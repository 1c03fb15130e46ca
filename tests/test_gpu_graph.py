"""phmm_forward_batch_graph: the asynchronous pass captured into a HIP graph
and replayed.  Every replay must be bit-identical to the stream launches of
phmm_forward_batch_async on the same inputs: replays of one key several times
with other work and synchronisations between them, new contents in the same
buffers (no new capture), a second batch of the same launch shape (the graph
updated in place) and one of another shape (a new graph), small batches
(one narrow class, capped grids) and large ones, long pairs included."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import paper_2606_25738_amd as phmm  # noqa: E402
import synth  # noqa: E402
from test_zz_no_alloc import concat, long_pairs  # noqa: E402

pytestmark = pytest.mark.gpu


class Buffers:
    def __init__(self, ctx, db):
        import torch
        n = db.n_pairs
        self.db = db
        self.out = torch.empty(n, dtype=torch.float64, device="cuda:0")
        self.fl = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        self.ws = torch.empty(phmm.phmm_workspace_bytes(ctx, n, db.max_read_len, db.max_hap_len),
                              dtype=torch.uint8, device="cuda:0")

    def run(self, ctx, fn, stream):
        self.out.fill_(float("nan"))
        self.fl.zero_()
        fn(ctx, self.db, self.out, self.fl, self.ws, stream)
        stream.synchronize()
        return self.out.cpu().numpy(), self.fl.cpu().numpy()


def same(a, b):
    return np.array_equal(a[0].view(np.uint64), b[0].view(np.uint64)) and np.array_equal(a[1], b[1])


def test_graph_replays_equal_stream_launches():
    import torch
    s = torch.cuda.Stream()
    big = concat(synth.generate("batched_uneven", 3, 50), long_pairs(5))
    small = synth.generate("batched_uneven", 8, 6)
    with phmm.Context() as c:
        for name, b in (("big", big), ("small", small)):
            buf = Buffers(c, phmm.DeviceBatch(b))
            want = buf.run(c, phmm.phmm_forward_batch_async, s)
            for rep in range(4):
                print("graph replay %d of the %s batch (%d pairs)" % (rep, name, buf.db.n_pairs), flush=True)
                got = buf.run(c, phmm.phmm_forward_batch_graph, s)
                assert same(got, want), "replay %d differs" % rep
                # eager work of the program between replays
                x = torch.randn(1 << 20, device="cuda:0")
                torch.cuda.synchronize()
                assert float((x * 2).sum()) == pytest.approx(2 * float(x.sum()), rel=1e-4)
            n = buf.db.n_pairs
            idx = np.concatenate([np.arange(0, n - 3, max(1, n // 100)), np.arange(max(0, n - 3), n)])
            ref = oracle.forward_pairs(b, idx, rescale=True)
            is32 = (want[1][idx] & phmm.PHMM_FLAG_FP32) != 0
            d = np.abs(want[0][idx] - ref)
            assert d[is32].max(initial=0) <= 1e-4 and d[~is32].max(initial=0) <= 1e-10


def test_graph_new_contents_same_buffers_and_shape_changes():
    """The graph reads the batch through its pointers: new bytes in the same
    device buffers replay without a new capture and give the new results; a
    second batch of the same size (other buffers: an in-place update of the
    graph's kernel parameters) and a batch of another size (a new graph) are
    each bit-identical to stream launches."""
    import torch
    s = torch.cuda.Stream()
    a = synth.generate("batched_uneven", 20, 40)
    with phmm.Context() as c:
        buf = Buffers(c, phmm.DeviceBatch(a))
        first = buf.run(c, phmm.phmm_forward_batch_graph, s)
        # other base qualities, same shapes, copied into the same buffers
        a2 = dict(a, base_quals=np.ascontiguousarray((a["base_quals"].astype(np.int64) * 7 + 3) % 41 + 2).astype(np.uint8))
        buf.db.t["base_quals"].copy_(torch.from_numpy(a2["base_quals"]))
        torch.cuda.synchronize()
        got = buf.run(c, phmm.phmm_forward_batch_graph, s)
        want = buf.run(c, phmm.phmm_forward_batch_async, s)
        assert same(got, want) and not same(got, first)
        # a second batch in other buffers with the same launch shape
        buf2 = Buffers(c, phmm.DeviceBatch(a2))
        assert same(buf2.run(c, phmm.phmm_forward_batch_graph, s), want)
        # another size, then back to the first buffers
        b = synth.generate("genome_scale", 4, 30)
        buf3 = Buffers(c, phmm.DeviceBatch(b))
        assert same(buf3.run(c, phmm.phmm_forward_batch_graph, s),
                    buf3.run(c, phmm.phmm_forward_batch_async, s))
        assert same(buf.run(c, phmm.phmm_forward_batch_graph, s), want)
        for _ in range(3):  # more keys than the context keeps graphs for
            for bb in (buf, buf2, buf3):
                bb.run(c, phmm.phmm_forward_batch_graph, s)
        assert same(buf.run(c, phmm.phmm_forward_batch_graph, s), want)
