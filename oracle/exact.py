"""Exact references used to pin the C oracle on tiny inputs (test only).

Both functions below work from the *path model* of the PairHMM (paper,
Section 2): a read is explained by a path of hidden states M (read base
aligned to a haplotype base), I (read base inserted) and D (haplotype base
skipped).  The transition weights are the push-form reading of eq.2:

  start  : M(1, j0+1) for j0 = 0..k-1 with weight (1/k) T_DM_1 P(r_1|h_{j0+1})
           (the D(0, j) = C/k start row of eq.1 with C removed)
  M(i,j) -> M(i+1,j+1)  T_MM_{i+1} P(r_{i+1}|h_{j+1})
  I(i,j) -> M(i+1,j+1)  T_IM_{i+1} P(r_{i+1}|h_{j+1})
  D(i,j) -> M(i+1,j+1)  T_DM_{i+1} P(r_{i+1}|h_{j+1})
  M(i,j) -> I(i+1,j)    T_MI_{i+1}
  I(i,j) -> I(i+1,j)    T_II_{i+1}
  M(i,j) -> D(i,j+1)    T_MD_i
  D(i,j) -> D(i,j+1)    T_DD_i
  end    : the path stops on first entering row l in M or I (eq.4)

``brute_force`` enumerates every path one by one (exponential; l, k <= 6).
``dag_sum`` sums the same path weights exactly over the state DAG with
``fractions.Fraction`` (polynomial; l, k <= ~30).  Neither evaluates the
pull-form recurrences of eq.2 that the C oracle uses.
"""
from __future__ import annotations

from fractions import Fraction

PM, PX, TMM, TIM, TDM, TMI, TII, TMD, TDD = range(9)


def _match(r: int, h: int) -> bool:
    n = ord("N")
    return r == h or r == n or h == n


def _emit(pri, i, read, hap, j):
    """P(r_i | h_j) with 1-based i, j (eq.3)."""
    row = pri[i - 1]
    return row[PM] if _match(read[i - 1], hap[j - 1]) else row[PX]


def _edges(pri, read, hap, state):
    """Outgoing (next_state, weight) of a state (kind, i, j)."""
    l, k = len(read), len(hap)
    kind, i, j = state
    out = []
    if kind in ("M", "I") and i == l:
        return out  # absorbed at the last row
    if i < l and j + 1 <= k:
        w = {"M": TMM, "I": TIM, "D": TDM}[kind]
        out.append((("M", i + 1, j + 1), pri[i][w] * _emit(pri, i + 1, read, hap, j + 1)))
    if kind in ("M", "I") and i < l:
        w = TMI if kind == "M" else TII
        out.append((("I", i + 1, j), pri[i][w]))
    if kind in ("M", "D") and j + 1 <= k:
        w = TMD if kind == "M" else TDD
        out.append((("D", i, j + 1), pri[i - 1][w]))
    return out


def _starts(pri, read, hap, one):
    k = len(hap)
    out = []
    for j0 in range(k):
        w = one / k * pri[0][TDM] * _emit(pri, 1, read, hap, j0 + 1)
        out.append((("M", 1, j0 + 1), w))
    return out


def _is_end(state, l):
    return state[0] in ("M", "I") and state[1] == l


def brute_force(pri, read: bytes, hap: bytes) -> float:
    """Sum of all path weights by explicit enumeration (float)."""
    read = bytes(read)
    hap = bytes(hap)
    l = len(read)
    total = 0.0
    stack = [(s, w) for s, w in _starts(pri, read, hap, 1.0)]
    while stack:
        s, w = stack.pop()
        if _is_end(s, l):
            total += w
            continue
        for t, tw in _edges(pri, read, hap, s):
            stack.append((t, w * tw))
    return total


def count_paths(read_len: int, hap_len: int) -> int:
    """Number of complete paths (used to show the enumeration is not empty)."""
    pri = [[1] * 9 for _ in range(read_len)]
    read = b"A" * read_len
    hap = b"A" * hap_len
    n = 0
    stack = [s for s, _ in _starts(pri, read, hap, Fraction(1))]
    while stack:
        s = stack.pop()
        if _is_end(s, read_len):
            n += 1
            continue
        stack.extend(t for t, _ in _edges(pri, read, hap, s))
    return n


def dag_sum(pri, read: bytes, hap: bytes):
    """Exact sum of all path weights over the state DAG.

    ``pri`` entries may be Fractions (exact) or floats.  States are visited
    in an order where every edge goes forward: rows increase, and inside a
    row D(i, j) follows M(i, j-1) and D(i, j-1)."""
    read = bytes(read)
    hap = bytes(hap)
    l, k = len(read), len(hap)
    one = Fraction(1) if isinstance(pri[0][0], Fraction) else 1.0
    acc = {}
    for s, w in _starts(pri, read, hap, one):
        acc[s] = acc.get(s, 0) + w
    total = 0
    for i in range(1, l + 1):
        for j in range(1, k + 1):
            for kind in ("M", "I", "D"):
                s = (kind, i, j)
                w = acc.pop(s, None)
                if w is None:
                    continue
                if _is_end(s, l):
                    total += w
                    continue
                for t, tw in _edges(pri, read, hap, s):
                    acc[t] = acc.get(t, 0) + w * tw
    return total


def path_weight(pri, read: bytes, hap: bytes, cols) -> float | None:
    """Weight of one alignment path given, for every read base, the 1-based
    haplotype column it is aligned to (M), or 0 for an inserted base (I).
    Deletions are the column jumps between consecutive aligned bases.
    Returns None when the path is not a path of the model."""
    read = bytes(read)
    hap = bytes(hap)
    l = len(read)
    if len(cols) != l or cols[0] <= 0:
        return None
    w = 1.0 / len(hap) * pri[0][TDM] * _emit(pri, 1, read, hap, cols[0])
    state = ("M", 1, cols[0])
    for i in range(2, l + 1):
        c = cols[i - 1]
        kind, _, j = state
        if c == 0:  # insertion keeps the column
            if kind == "D":
                return None
            w *= pri[i - 1][TMI if kind == "M" else TII]
            state = ("I", i, j)
            continue
        if c <= j:
            return None
        gap = c - j - 1
        if gap > 0:
            if kind != "M":
                return None
            w *= pri[i - 2][TMD] * pri[i - 2][TDD] ** (gap - 1)
            kind = "D"
        w *= pri[i - 1][{"M": TMM, "I": TIM, "D": TDM}[kind]] * _emit(pri, i, read, hap, c)
        state = ("M", i, c)
    return w
