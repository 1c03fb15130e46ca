"""Host-side model of the library's launch protocol, for CPU tests.

It follows the device code's control flow and index arithmetic, not its
floating point: the packer (runs, per-class greedy sizing, class choice,
unrelated-haplotype routing, segment scan, emission), the queues between the
kernel families (deferred packs, FP64 rerun items, the FP64 hand-off of
underflowed pairs to the long list) and the long kernel's ring protocol
between tiles (slot take-over, producer/consumer windows, ring back-pressure,
final sums), run as a discrete-event simulation over a given number of
resident wavefronts.  Every array index the kernels form is checked against
the capacity the host allocates, every persistent loop is walked to its exit,
and a long-kernel schedule that stops making progress is reported as a
deadlock.  Which pairs FP32 rejects, or FP64 finds underflowed, is an input
(a predicate per pair), so both the predicted path and the worst case
(everything rejected, everything handed to the long kernel) can be checked.
"""
from __future__ import annotations

import numpy as np

NUM_CLASSES = 21
WAVE = 64
MAX_N = 24
SHORT_MAX_COLS = WAVE * MAX_N
MAX_PAIRS_PER_PACK = 32
CHUNK = 256
SMALL_BATCH_PAIRS = 8192
SC_MAX_INS_Q = 65
RING = 512
LONG_TILE = 16 * WAVE
LONG_FP32_MAX_GAP = 10  # FP32 long pairs need every gap byte at most this
KMER_BASES = 32


def class_n(c: int) -> int:
    return 4 + c


class ModelError(AssertionError):
    pass


def need(cond: bool, what: str):
    if not cond:
        raise ModelError(what)


def long_active_waves(tiles: int, g: int) -> int:
    """Wavefronts of a long-kernel grid of g that take tiles: the first
    `tiles` when there are fewer tiles than wavefronts, else all."""
    return tiles if 0 < tiles < g else g


class Policy:
    def __init__(self, precision=0, force_class=-1, one_pair_per_wave=False, fp32_max_rows=1024,
                 long_fp32_max_rows=0, route_diverse=True, cost=None):
        self.precision = precision
        self.force_class = force_class
        self.one_pair_per_wave = one_pair_per_wave
        self.fp32_max_rows = fp32_max_rows
        self.long_fp32_max_rows = long_fp32_max_rows
        self.route_diverse = route_diverse
        self.long_haps = True  # the batch's haplotype bound admits long pairs
        self.cost = cost if cost is not None else [[class_n(c) + 3.0 for c in range(NUM_CLASSES)]
                                                   for _ in range(2)]

    def for_batch(self, n_pairs: int, max_hap_len: int) -> "Policy":
        """A small batch is packed in the narrowest class that holds its
        longest short haplotype unless a class is forced."""
        p = Policy(self.precision, self.force_class, self.one_pair_per_wave, self.fp32_max_rows,
                   self.long_fp32_max_rows, self.route_diverse, self.cost)
        if n_pairs <= SMALL_BATCH_PAIRS and p.force_class < 0:
            k = max(1, min(max_hap_len, SHORT_MAX_COLS))
            n = max(class_n(0), (k + WAVE - 1) // WAVE)
            p.force_class = min(n, MAX_N) - 4
        p.long_haps = max_hap_len > SHORT_MAX_COLS
        return p


def _kmer_set(h: bytes) -> set:
    n = min(len(h), KMER_BASES)
    code, out = 0, set()
    for j in range(n):
        code = ((code << 2) | ((h[j] >> 1) & 3)) & 255
        if j >= 3:
            out.add(code)
    return out


def _similar(a: set, b: set) -> bool:
    return 2 * len(a & b) >= len(a | b)


class LaunchModel:
    """One call of the forward pass on a host batch (the dict the binding
    takes), under policy `pol` (already specialised for the batch)."""

    def __init__(self, batch, pol: Policy):
        self.b = batch
        self.pol = pol
        self.pl = np.asarray(batch["pair_list"], np.int64).reshape(-1, 2)
        self.n = len(self.pl)
        ro, ho = batch["read_offsets"].astype(np.int64), batch["hap_offsets"].astype(np.int64)
        self.rlen = np.diff(ro)
        self.hlen = np.diff(ho)
        self.ro, self.ho = ro, ho
        cap = max(self.n, 1)
        self.cap = cap  # every per-pair array of the workspace holds n_pairs entries
        # long lists q = 2 * precision + general (general: the read has
        # several gap bytes, a gap byte 0 or an insertion byte over 65)
        self.long_list = [[], [], [], []]
        self.long_pend = [[], []]  # per precision, before routing
        self.bound_error = False   # a long pair in a batch whose bound says none
        self.out_writes = np.zeros(self.n, np.int64)
        self.flags = np.zeros(self.n, np.int64)

    # ---------------------------------------------------------------- packer
    def k_of(self, q):
        return int(self.hlen[self.pl[q, 1]])

    def runs(self):
        starts = [p for p in range(self.n)
                  if p == 0 or self.pl[p, 0] != self.pl[p - 1, 0] or p % CHUNK == 0]
        for p in starts:
            e = p + 1
            while e < self.n and self.pl[e, 0] == self.pl[p, 0] and e % CHUNK != 0:
                e += 1
            yield p, e

    def pack(self):
        pol = self.pol
        self.info = {}
        seg_cnt = np.zeros((2, NUM_CLASSES), np.int64)
        for p, e in self.runs():
            need(e <= self.n and e > p, "run bounds")
            l = int(self.rlen[self.pl[p, 0]])
            prec = 1 if (pol.precision == 1 or l > pol.fp32_max_rows) else 0
            lprec = 1 if (pol.precision == 1 or l > pol.long_fp32_max_rows) else 0
            packs = [0] * NUM_CLASSES
            used = [WAVE] * NUM_CLASSES
            np_ = [0] * NUM_CLASSES
            fits = [True] * NUM_CLASSES
            nshort = 0
            for q in range(p, e):
                k = self.k_of(q)
                if k > SHORT_MAX_COLS:
                    if pol.long_haps:
                        self.long_pend[lprec].append(q)
                        need(len(self.long_pend[lprec]) <= self.cap, "pending long list overflow")
                    else:
                        self.bound_error = True
                        self.long_list[3].append(q)
                        need(len(self.long_list[3]) <= self.cap, "long list overflow")
                    used = [WAVE] * NUM_CLASSES
                    np_ = [0] * NUM_CLASSES
                    continue
                nshort += 1
                for c in range(NUM_CLASSES):
                    sl = -(-k // class_n(c))
                    if sl > WAVE:
                        fits[c] = False
                        continue
                    if pol.one_pair_per_wave or used[c] + sl > WAVE or np_[c] == MAX_PAIRS_PER_PACK:
                        packs[c] += 1
                        used[c] = 0
                        np_[c] = 0
                    used[c] += sl
                    np_[c] += 1
            if prec == 0 and pol.route_diverse and e - p >= 2:
                sets = []
                for q in range(p, e):
                    k = self.k_of(q)
                    if k > SHORT_MAX_COLS or k < 8:
                        continue
                    h = self.b["haplotypes"][self.ho[self.pl[q, 1]]:self.ho[self.pl[q, 1] + 1]]
                    sets.append(_kmer_set(bytes(h)))
                    if len(sets) == 4:
                        break
                if len(sets) >= 2 and not any(_similar(sets[0], s) for s in sets[1:]):
                    prec = 1
            info = None
            if nshort > 0:
                best, best_cost = -1, 3.0e38
                for c in range(NUM_CLASSES):
                    if not fits[c] or (pol.force_class >= 0 and c != pol.force_class):
                        continue
                    v = packs[c] * pol.cost[prec][c]
                    if v < best_cost:
                        best, best_cost = c, v
                if best < 0:
                    best = NUM_CLASSES - 1
                need(fits[best], "chosen class %d does not hold a pair of run %d" % (best, p))
                need(packs[best] < (1 << 24), "pack count overflows the run info word")
                info = (best, prec, packs[best])
                seg_cnt[prec, best] += packs[best]
            self.info[p] = info
        self.pack_cnt = seg_cnt
        self.pack_base = np.zeros_like(seg_cnt)
        acc = 0
        for prec in range(2):
            for c in range(NUM_CLASSES):
                self.pack_base[prec, c] = acc
                acc += seg_cnt[prec, c]
        need(acc <= self.cap, "pack array overflow: %d packs for %d entries" % (acc, self.cap))
        self.item_base = np.concatenate([[0], np.cumsum(seg_cnt[0])[:-1]])
        # emission
        self.packs = [None] * acc
        fill = np.zeros((2, NUM_CLASSES), np.int64)
        for p, e in self.runs():
            info = self.info[p]
            if info is None:
                continue
            c, prec, npk = info
            slot = self.pack_base[prec, c] + fill[prec, c]
            fill[prec, c] += npk
            N = class_n(c)
            written, used, np_, start = 0, WAVE, 0, p
            out = []
            for q in range(p, e):
                k = self.k_of(q)
                if k > SHORT_MAX_COLS:
                    if np_:
                        out.append((start, np_))
                    used, np_ = WAVE, 0
                    continue
                sl = -(-k // N)
                if self.pol.one_pair_per_wave or used + sl > WAVE or np_ == MAX_PAIRS_PER_PACK:
                    if np_:
                        out.append((start, np_))
                    used, np_, start = 0, 0, q
                used += sl
                np_ += 1
            if np_:
                out.append((start, np_))
            need(len(out) == npk, "run %d: emit wrote %d packs, count sized %d" % (p, len(out), npk))
            for j, pk in enumerate(out):
                need(0 <= slot + j < acc, "pack slot out of range")
                need(self.packs[slot + j] is None, "pack slot written twice")
                self.packs[slot + j] = (c, prec) + pk
        need(all(x is not None for x in self.packs), "pack slot never written")
        # every short pair in exactly one pack, packs hold one read
        seen = np.zeros(self.n, np.int64)
        for c, prec, start, npairs in self.packs:
            need(1 <= npairs <= MAX_PAIRS_PER_PACK, "pack pair count")
            lanes = 0
            for q in range(start, start + npairs):
                need(q < self.n and self.pl[q, 0] == self.pl[start, 0], "pack crosses reads")
                k = self.k_of(q)
                need(k <= SHORT_MAX_COLS, "long pair in a pack")
                lanes += -(-k // class_n(c))
                seen[q] += 1
            need(lanes <= WAVE, "pack of %d lanes" % lanes)
        for q in range(self.n):
            need(seen[q] == (0 if self.k_of(q) > SHORT_MAX_COLS else 1), "pair %d packed %d times"
                 % (q, seen[q]))

    # ---------------------------------------------------------------- short kernels
    def _segments(self, c, start, mask):
        """Lane layout of a pack (first lane, lanes) per computed pair, and the
        LDS indices the result step reads."""
        N = class_n(c)
        segs, first = [], 0
        for s in range(32):
            if mask >> s & 1:
                k = self.k_of(start + s)
                lanes = -(-k // N)
                segs.append((start + s, s, first, lanes))
                first += lanes
        need(first <= WAVE, "segments of %d lanes" % first)
        for _, _, f, cnt in segs:
            need(0 <= f and f + cnt <= WAVE, "segment lanes outside the wavefront")
        return segs

    def route(self):
        """The routing kernel: each pending long pair goes to the lean list
        of its precision when its read has one gap byte (>= 1) and insertion
        bytes the scaled row form allows, else to the general one; an FP32
        pair whose read has a gap byte above 10 goes to the FP64 lists."""
        for prec in (0, 1):
            for q in self.long_pend[prec]:
                varying, sc_ok = self._read_profile(q)
                r = self.pl[q, 0]
                wide = prec == 1 or bool((self.b["gcp"][self.ro[r]:self.ro[r + 1]] > LONG_FP32_MAX_GAP).any())
                lq = 2 * (1 if wide else 0) + (0 if (sc_ok and not varying) else 1)
                self.long_list[lq].append(q)
                need(len(self.long_list[lq]) <= self.cap, "long list overflow")

    def _read_profile(self, start):
        r = self.pl[start, 0]
        a, b = self.ro[r], self.ro[r + 1]
        g = self.b["gcp"][a:b]
        i = self.b["ins_quals"][a:b]
        varying = bool((g != g[0]).any())
        sc_ok = not bool(((g == 0) | (i > SC_MAX_INS_Q)).any())
        return varying, sc_ok

    def run(self, accept32, ok64, grids=(None, None)):
        """Walks every kernel family in the order the passes launch them.
        accept32(pair) / ok64(pair): whether the FP32 sum passes the threshold
        and whether the FP64 sum is above the hand-off bound."""
        self.pack()
        if self.pol.long_haps:
            self.route()
        defer = [[] for _ in range(NUM_CLASSES)]
        items = [[] for _ in range(NUM_CLASSES)]
        if self.pol.precision == 0:
            for c in range(NUM_CLASSES):
                for it in range(self.pack_cnt[0, c]):
                    gi = self.pack_base[0, c] + it
                    _, _, start, npairs = self.packs[gi]
                    varying, sc_ok = self._read_profile(start)
                    if varying or not sc_ok:
                        defer[c].append(gi)
                        need(len(defer[c]) <= self.pack_cnt[0, c], "deferred queue overflow")
                        continue
                    self._fp32_pack(c, gi, (1 << npairs) - 1, accept32, items)
            for c in range(NUM_CLASSES):
                for gi in defer[c]:
                    _, _, start, npairs = self.packs[gi]
                    self._fp32_pack(c, gi, (1 << npairs) - 1, accept32, items)
        for c in range(NUM_CLASSES):
            work = [(self.pack_base[1, c] + it, None) for it in range(self.pack_cnt[1, c])]
            work += [(gi, m) for gi, m in items[c]]
            for gi, m in work:
                _, _, start, npairs = self.packs[gi]
                mask = (1 << npairs) - 1 if m is None else m
                for pair, off, f, cnt in self._segments(c, start, mask):
                    if ok64(pair):
                        self._write(pair, 0x12 if m is not None else 0x10)
                    else:
                        self.long_list[3].append(pair)
                        need(len(self.long_list[3]) <= self.cap, "FP64 long list overflow")
        for which in range(4):
            if self.long_list[which]:
                self.long_protocol(which, grids[which // 2])
                for pair in self.long_list[which]:
                    self._write(pair, 0x0c | (0x01 if which < 2 else 0x10))
        for q in range(self.n):
            need(self.out_writes[q] == 1, "pair %d written %d times" % (q, self.out_writes[q]))
        return self.flags

    def _fp32_pack(self, c, gi, mask, accept32, items):
        _, _, start, npairs = self.packs[gi]
        rej = 0
        for pair, off, f, cnt in self._segments(c, start, mask):
            if accept32(pair):
                self._write(pair, 0x01)
            else:
                rej |= 1 << off
        if rej:
            items[c].append((gi, rej))
            need(len(items[c]) <= self.pack_cnt[0, c], "rerun item queue overflow")

    def _write(self, pair, flag):
        self.out_writes[pair] += 1
        self.flags[pair] = flag

    # ---------------------------------------------------------------- long kernel
    def long_protocol(self, which, grid, max_events=10_000_000):
        """Discrete-event run of the long kernel's tile pipeline with `grid`
        resident wavefronts (default: the persistent grid of a full chip)."""
        lst = self.long_list[which]
        tiles = [-(-self.k_of(q) // LONG_TILE) for q in lst]
        pref = np.concatenate([[0], np.cumsum(tiles)]).astype(np.int64)
        total = int(pref[-1])
        grid = grid or 1024
        nslot = 2 * grid
        active = long_active_waves(total, grid)
        need(active <= grid, "active wavefronts within the grid")
        done = [0] * nslot
        owner = [0] * nslot
        prog = [0] * nslot
        published = [0] * nslot   # rows of the slot's ring written this lap set
        fin = [False] * nslot
        cursor = 0

        class Wave:
            pass

        waves = []
        for _ in range(active):
            w = Wave()
            w.state = "claim"
            waves.append(w)

        def item_of(it):
            s = int(np.searchsorted(pref, it, side="right") - 1)
            need(0 <= s < len(lst) and pref[s] <= it < pref[s + 1], "tile item lookup")
            return s, it - int(pref[s]), tiles[s]

        events = 0
        finished = 0
        while True:
            progress = False
            for w in waves:
                while True:
                    events += 1
                    need(events < max_events, "long kernel model did not finish")
                    if w.state == "claim":
                        it = cursor
                        cursor += 1
                        if it >= total:
                            w.state = "exit"
                            progress = True
                            break
                        s, tile, nt = item_of(it)
                        w.it, w.tile, w.nt = it, tile, nt
                        w.l = int(self.rlen[self.pl[lst[s], 0]])
                        w.prod, w.cons = tile > 0, tile + 1 < nt
                        w.slot, w.pslot = it % nslot, (it + nslot - 1) % nslot
                        w.state = "takeover"
                        progress = True
                    elif w.state == "takeover":
                        if w.it >= nslot and done[w.slot] != w.it - nslot + 1:
                            break
                        if w.cons:
                            published[w.slot] = 0
                            fin[w.slot] = False
                            prog[w.slot] = 0
                            owner[w.slot] = w.it + 1
                        else:
                            done[w.slot] = w.it + 1
                        w.state = "wait_owner"
                        progress = True
                    elif w.state == "wait_owner":
                        if w.prod and owner[w.pslot] != w.it:
                            break
                        w.i0, w.row = 0, 0
                        w.state = "window"
                        progress = True
                    elif w.state == "window":
                        if w.i0 >= w.l:
                            w.state = "final"
                            progress = True
                            continue
                        nrows = min(WAVE, w.l - w.i0)
                        if w.prod:
                            prog[w.pslot] = w.i0
                            if published[w.pslot] < w.i0 + nrows:
                                break
                        w.row = w.i0
                        w.end = w.i0 + nrows
                        w.state = "rows"
                        progress = True
                    elif w.state == "rows":
                        i = w.row
                        if w.cons and i >= RING and prog[w.slot] < i - RING + 1:
                            break
                        if w.cons:
                            published[w.slot] = i + 1
                        w.row += 1
                        progress = True
                        if w.row >= w.end:
                            w.i0 += WAVE
                            w.state = "window"
                    elif w.state == "final":
                        if w.prod:
                            if not fin[w.pslot]:
                                break
                            done[w.pslot] = w.it
                        if w.cons:
                            fin[w.slot] = True
                        finished += 1
                        w.state = "claim"
                        progress = True
                    else:
                        break
            if all(w.state == "exit" for w in waves):
                break
            if not progress:
                stuck = [(w.state, getattr(w, "it", None)) for w in waves if w.state != "exit"]
                raise ModelError("long kernel deadlock with %d resident waves: %s"
                                 % (grid, stuck[:8]))
        need(finished == total, "long kernel finished %d of %d tiles" % (finished, total))
        return total
