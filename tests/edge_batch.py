"""Hand-built batches shared by the GPU parity tests and the CPU model of the
launch protocol: make_batch() turns (read, hap, quals...) tuples into the
binding's batch dict, edge_pairs() lists the degenerate inputs of the method
(one-base reads and haplotypes, 'N' bases, Phred 0 and 255, haplotypes at the
wavefront's column limits, per-row gap penalties)."""
import numpy as np


def make_batch(pairs):
    """pairs: list of (read, hap, bq, iq, dq, gq) with bytes / int arrays;
    one read and one haplotype per pair."""
    reads, haps, bq, iq, dq, gq, ro, ho, pl = [], [], [], [], [], [], [0], [0], []
    for r, h, q, i, d, g in pairs:
        reads.append(np.frombuffer(r, np.uint8))
        haps.append(np.frombuffer(h, np.uint8))
        for lst, v in ((bq, q), (iq, i), (dq, d), (gq, g)):
            lst.append(np.broadcast_to(np.asarray(v, np.uint8), (len(r),)))
        ro.append(ro[-1] + len(r))
        ho.append(ho[-1] + len(h))
        pl.append((len(ro) - 2, len(ho) - 2))
    cat = lambda x: np.ascontiguousarray(np.concatenate(x).astype(np.uint8))
    return dict(reads=cat(reads), base_quals=cat(bq), ins_quals=cat(iq), del_quals=cat(dq),
                gcp=cat(gq), read_offsets=np.array(ro, np.uint64),
                haplotypes=cat(haps), hap_offsets=np.array(ho, np.uint64),
                pair_list=np.array(pl, np.uint32))


def rnd(rng, n, alpha=b"ACGT"):
    a = np.frombuffer(alpha, np.uint8)
    return bytes(a[rng.integers(0, len(a), n)])


def edge_pairs():
    rng = np.random.default_rng(5)
    src = rnd(rng, 3000)
    return [
        (b"A", b"A", 30, 45, 45, 10),
        (b"A", b"C", 30, 45, 45, 10),
        (b"ACGT", b"A", 20, 45, 45, 10),
        (b"A", rnd(rng, 97), 20, 45, 45, 10),
        (b"N" * 30, rnd(rng, 50), 20, 45, 45, 10),
        (rnd(rng, 30), b"N" * 40, 20, 45, 45, 10),
        (rnd(rng, 40, b"ACGTN"), rnd(rng, 60, b"ACGTN"), 25, 40, 40, 10),
        (src[100:250], src[90:90 + 64 * 4], 30, 45, 45, 10),           # exactly 64 lanes x 4
        (src[100:250], src[90:90 + 64 * 24], 30, 45, 45, 10),          # widest short pair
        (src[100:250], src[90:90 + 64 * 24 + 1], 30, 45, 45, 10),      # first long pair
        (src[0:150], src[0:150], 0, 0, 0, 0),                           # Phred 0 everywhere
        (src[0:150], src[0:150], 255, 255, 255, 255),                   # Phred 255 everywhere
        (src[5:120], src[0:300], np.arange(115) % 60, 30, 30, np.arange(115) % 40 + 1),
    ]
