"""Genotype likelihoods on the GPU (phmm_genotype_batch and its
stream-ordered form) against the FP64 oracle of the genotyping step, on
synthetic likelihood matrices and on the PairHMM output of real batches.

Tolerance: both sides evaluate each read's term in FP64 (the library as
max + log10(1 + 10^-d) - log10 2, the oracle as the plain two-term sum with
10^max factored out); each term differs by a few units in the last place of
its magnitude, so a region's GL agrees within 1e-12 relative (plus 1e-12
absolute).  The best genotype is compared where the oracle's maximum is
unique by more than the tolerance, and checked to be a maximum otherwise."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import paper_2606_25738_amd as phmm  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

RTOL = 1e-12
ATOL = 1e-12
NONE = 0xFFFFFFFF


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = phmm.Context()
    yield c
    c.close()


def tol(gl_ref, extra=0.0):
    return RTOL * np.abs(gl_ref) + ATOL + extra


def check_regions(gl, go, best, regions, gls_ref, best_ref, R, extra_per_read=0.0):
    for k, g in enumerate(regions):
        ref = gls_ref[k]
        got = gl[int(go[g]):int(go[g]) + len(ref)]
        t = tol(ref, extra_per_read * int(R[g]))
        bad = np.abs(got - ref) > t
        assert not bad.any(), "region %d genotype %d: %r vs %r" % (
            g, int(np.argmax(bad)), got[bad][:3], ref[bad][:3])
        b = int(best[g])
        assert 0 <= b < len(ref), (g, b)
        top = np.sort(ref)[::-1]
        if len(ref) == 1 or top[0] - top[1] > 2 * t.max():
            assert b == best_ref[k], (g, b, best_ref[k])
        else:
            assert ref[b] >= top[0] - 2 * t.max(), (g, b)


def sample_regions(R, H, n, seed):
    """Extremes (largest H, largest R, no reads, one haplotype) plus random regions."""
    rng = np.random.default_rng(seed)
    pick = {int(np.argmax(H)), int(np.argmax(R)), int(np.argmax(R * H))}
    for cond in (R == 0, H == 1):
        if cond.any():
            pick.add(int(np.flatnonzero(cond)[0]))
    pick.update(rng.choice(len(R), size=min(n, len(R)), replace=False).tolist())
    return sorted(pick)


def test_host_form_matches_oracle(ctx):
    # H up to 40 (820 genotypes: 13 lane passes), R up to 120 (LDS chunks of
    # 1024 // H reads with a ragged last chunk), 10% long-read values
    lk, lo, R, H = synth.genotype_lk(11, 400, reads=(0, 120), haps=(1, 40), long_frac=0.1)
    say("genotype host form: 400 regions, %d likelihoods" % lk.size)
    gl, best = phmm.phmm_genotype_batch(ctx, lk, lo, R, H)
    go, n_gl = phmm.genotype_offsets(H)
    assert gl.size == n_gl
    regs = sample_regions(R, H, 50, 0)
    gls, bref = oracle.genotype_batch(lk, lo, R, H, regs)
    check_regions(gl, go, best, regs, gls, bref, R)
    # homozygous entries are plain sums of the read's values: the same sum
    for g in regs:
        r, h, o = int(R[g]), int(H[g]), int(lo[g])
        m = lk[o:o + r * h].reshape(r, h)
        for a in range(h):
            assert abs(gl[int(go[g]) + a * (a + 3) // 2] - m[:, a].sum()) <= tol(m[:, a].sum())


def test_async_form_and_offsets_with_gaps(ctx):
    import torch
    lk, lo, R, H = synth.genotype_lk(12, 300, reads=(0, 70), haps=(1, 24))
    go, n_gl = phmm.genotype_offsets(H)
    go = go + 3 * np.arange(300, dtype=np.uint64)  # gaps of 3 between the blocks
    fill = np.full(n_gl + 3 * 300, 7.0)
    gl_h, best_h = phmm.phmm_genotype_batch(ctx, lk, lo, R, H, gl_offsets=go, gl=fill.copy())
    dev = "cuda:0"
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to(dev)
    d_gl = torch.full((fill.size,), 7.0, dtype=torch.float64, device=dev)
    d_best = torch.empty(300, dtype=torch.int32, device=dev)
    s = torch.cuda.Stream()
    args = (t(lk, np.float64), t(lo, np.int64), t(R, np.int32), t(H, np.int32), t(go, np.int64))
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        phmm.phmm_genotype_batch_async(ctx, *args, d_gl, d_best, s)
    s.synchronize()
    gl_d = d_gl.cpu().numpy()
    np.testing.assert_array_equal(gl_d, gl_h)
    np.testing.assert_array_equal(d_best.cpu().numpy().view(np.uint32), best_h)
    gaps = np.ones(fill.size, bool)
    for g in range(300):
        gaps[int(go[g]):int(go[g]) + int(H[g]) * (int(H[g]) + 1) // 2] = False
    assert gaps.sum() == 900 and np.all(gl_h[gaps] == 7.0)
    regs = sample_regions(R, H, 40, 1)
    gls, bref = oracle.genotype_batch(lk, lo, R, H, regs)
    check_regions(gl_h, go, best_h, regs, gls, bref, R)


def test_async_form_skips_regions_outside_arrays(ctx):
    import torch
    lk, lo, R, H = synth.genotype_lk(13, 6, reads=(3, 9), haps=(2, 6))
    go, n_gl = phmm.genotype_offsets(H)
    gl_ref, best_ref = phmm.phmm_genotype_batch(ctx, lk, lo, R, H)
    lo2, H2, go2 = lo.copy(), H.copy(), go.copy()
    lo2[1] = lk.size - 1                 # matrix runs past n_lk
    go2[3] = n_gl - 1                    # genotype block runs past n_gl
    H2[4] = 0                            # no haplotypes
    dev = "cuda:0"
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to(dev)
    d_gl = torch.full((n_gl,), 7.0, dtype=torch.float64, device=dev)
    d_best = torch.zeros(6, dtype=torch.int32, device=dev)
    phmm.phmm_genotype_batch_async(ctx, t(lk, np.float64), t(lo2, np.int64), t(R, np.int32),
                                   t(H2, np.int32), t(go2, np.int64), d_gl, d_best, None)
    torch.cuda.synchronize()
    gl = d_gl.cpu().numpy()
    best = d_best.cpu().numpy().view(np.uint32)
    for g in range(6):
        blk = slice(int(go[g]), int(go[g]) + int(H[g]) * (int(H[g]) + 1) // 2)
        if g in (1, 3, 4):
            assert best[g] == NONE
            if g != 3:
                assert np.all(gl[blk] == 7.0)
        else:
            assert best[g] == best_ref[g]
            np.testing.assert_array_equal(gl[blk], gl_ref[blk])


def test_genotypes_of_the_pairhmm_output(ctx):
    """Forward pass on the GPU (FP32 with FP64 reruns), genotype call straight
    on its device output, against the oracle's forward pass and genotyping.
    Each read's term moves by at most the largest change of its two
    likelihoods, so GL agrees within 1e-4 per read (the FP32 tolerance)."""
    import torch
    b = synth.generate("batched_uneven", 0, 12)
    rp, rr, rh = b["region_pairs"], b["region_reads"], b["region_haps"]
    R, H = np.diff(rr).astype(np.uint32), np.diff(rh).astype(np.uint32)
    assert np.array_equal(np.diff(rp), R.astype(np.int64) * H)
    lo = rp[:-1].astype(np.uint64)
    n = len(b["pair_list"])
    say("forward + genotype: 12 regions, %d pairs" % n)
    db = phmm.DeviceBatch(b, "cuda:0")
    out = torch.empty(n, dtype=torch.float64, device="cuda:0")
    fl = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    ws = torch.empty(phmm.phmm_workspace_bytes(ctx, n, db.max_read_len, db.max_hap_len),
                     dtype=torch.uint8, device="cuda:0")
    go, n_gl = phmm.genotype_offsets(H)
    d_gl = torch.empty(n_gl, dtype=torch.float64, device="cuda:0")
    d_best = torch.empty(12, dtype=torch.int32, device="cuda:0")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to("cuda:0")
    s = torch.cuda.Stream()
    args = (t(lo, np.int64), t(R, np.int32), t(H, np.int32), t(go, np.int64))
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        phmm.phmm_forward_batch_async(ctx, db, out, fl, ws, s)
        phmm.phmm_genotype_batch_async(ctx, out, *args, d_gl, d_best, s)
    phmm.phmm_device_status(ctx, ws)
    s.synchronize()
    lk_ref = oracle.forward_pairs(b)
    assert np.max(np.abs(out.cpu().numpy() - lk_ref)) <= 1e-4
    gls, bref = oracle.genotype_batch(lk_ref, lo, R, H)
    check_regions(d_gl.cpu().numpy(), go, d_best.cpu().numpy().view(np.uint32), range(12), gls,
                  bref, R, extra_per_read=1e-4)


def test_genome_scale_sized_batch(ctx):
    """100,000 regions of 2-16 haplotypes and up to 80 reads, sampled
    against the oracle."""
    lk, lo, R, H = synth.genotype_lk(14, 100000, reads=(0, 80), haps=(2, 16))
    say("genotype: 100000 regions, %d likelihoods" % lk.size)
    gl, best = phmm.phmm_genotype_batch(ctx, lk, lo, R, H)
    go, _ = phmm.genotype_offsets(H)
    regs = sample_regions(R, H, 60, 2)
    gls, bref = oracle.genotype_batch(lk, lo, R, H, regs)
    check_regions(gl, go, best, regs, gls, bref, R)
