"""Independent textbook implementations used to pin the oracle (test-side only).

Nothing here is imported by the oracle or by the product.  Each function is a
plain restatement of a textbook definition, written without the antidiagonal
order, the pruning or the data structures that the oracle uses, so that the
two can only agree if the oracle is right:

* ``brute_seed_hits``    every (t, q) pair compared position by position;
* ``xdrop_closed_form``  ungapped extension with an unbounded X is the
                         maximum-sum prefix on each side;
* ``gotoh_extension``    full-matrix affine-gap extension DP from a corner
                         with a free end (the Y-drop DP with Y unbounded);
* ``gotoh_local``        Smith-Waterman with affine gaps (Gotoh);
* ``rescore`` / ``check_alignment``  invariants every alignment must satisfy.
"""
from __future__ import annotations

import numpy as np

NEG = -(1 << 30)


def care_offsets(pattern: str):
    return [i for i, c in enumerate(pattern) if c == "1"]


def brute_seed_hits(tc, ts, qc, qs, pattern, transitions=1, step=1):
    """Set of (t, q) with both windows valid and the care positions equal, or
    differing at exactly one position by a transition."""
    span = len(pattern)
    care = np.array(care_offsets(pattern))
    nt, nq = tc.shape[0], qc.shape[0]

    def valid(code, soft, n):
        bad = (code == 4) | (soft != 0)
        ok = []
        for p in range(0, n - span + 1):
            if not bad[p:p + span].any():
                ok.append(p)
        return np.array(ok, dtype=np.int64)

    tw = valid(tc, ts, nt)
    tw = tw[tw % step == 0]
    qw = valid(qc, qs, nq)
    if tw.shape[0] == 0 or qw.shape[0] == 0:
        return set()
    T = tc[tw[:, None] + care[None, :]].astype(np.int16)
    out = set()
    for s in range(0, qw.shape[0], 256):
        Q = qc[qw[s:s + 256, None] + care[None, :]].astype(np.int16)
        diff = T[None, :, :] != Q[:, None, :]
        nd = diff.sum(axis=2)
        trans = ((T[None, :, :] ^ Q[:, None, :]) == 2) & diff
        ok = nd == 0
        if transitions:
            ok |= (nd == 1) & (trans.sum(axis=2) == 1)
        qi, ti = np.nonzero(ok)
        for a, b in zip(qi, ti):
            out.add((int(tw[b]), int(qw[s + a])))
    return out


def xdrop_closed_form(tc, qc, t, q, span, sub):
    """Unbounded-X ungapped extension: on each side the extent is the shortest
    prefix attaining the maximum prefix sum (0 for the empty prefix)."""
    nt, nq = tc.shape[0], qc.shape[0]
    s0 = sum(sub[tc[t + u]][qc[q + u]] for u in range(span))
    right = [sub[tc[t + span - 1 + r]][qc[q + span - 1 + r]] for r in range(1, min(nt - t - span, nq - q - span) + 1)]
    left = [sub[tc[t - r]][qc[q - r]] for r in range(1, min(t, q) + 1)]

    def best(cols):
        pre = np.concatenate([[0], np.cumsum(cols)]) if cols else np.array([0])
        m = int(pre.max())
        return m, int(np.argmax(pre == m))

    bR, R = best(right)
    bL, L = best(left)
    return t - L, q - L, L + span + R, s0 + bL + bR


def gotoh_extension(A, B, sub, o, e):
    """Full-matrix extension DP from (0, 0) with a free end: H(0,0) = 0,
    E consumes B, F consumes A, a gap of length L costs o + L e.  Returns the
    matrices, the best score, the first (smallest i + j, then smallest i) cell
    attaining it, and the traceback (emission order) with diagonal > E > F in
    H and open > extend in gap states."""
    nA, nB = len(A), len(B)
    oe = o + e
    H = np.full((nA + 1, nB + 1), NEG, dtype=np.int64)
    E = np.full((nA + 1, nB + 1), NEG, dtype=np.int64)
    F = np.full((nA + 1, nB + 1), NEG, dtype=np.int64)
    G = np.full((nA + 1, nB + 1), NEG, dtype=np.int64)
    H[0, 0] = 0
    for i in range(nA + 1):
        for j in range(nB + 1):
            if i == 0 and j == 0:
                continue
            ev = max(H[i, j - 1] - oe, E[i, j - 1] - e) if j >= 1 else NEG
            fv = max(H[i - 1, j] - oe, F[i - 1, j] - e) if i >= 1 else NEG
            gv = H[i - 1, j - 1] + sub[A[i - 1]][B[j - 1]] if i >= 1 and j >= 1 else NEG
            E[i, j], F[i, j], G[i, j] = max(ev, NEG), max(fv, NEG), max(gv, NEG)
            H[i, j] = max(G[i, j], E[i, j], F[i, j])
    best = int(H.max())
    cand = [(i + j, i) for i, j in zip(*np.nonzero(H == best))]
    k, bi = min(cand)
    bj = k - bi
    ops = []
    i, j, state = bi, bj, 0
    while not (i == 0 and j == 0 and state == 0):
        if state == 0:
            if H[i, j] == G[i, j] and i >= 1 and j >= 1:
                ops.append(0)
                i, j = i - 1, j - 1
            elif H[i, j] == E[i, j]:
                state = 1
            else:
                state = 2
        elif state == 1:
            ops.append(1)
            if E[i, j] == H[i, j - 1] - oe:
                state = 0
            j -= 1
        else:
            ops.append(2)
            if F[i, j] == H[i - 1, j] - oe:
                state = 0
            i -= 1
    return best, bi, bj, ops


def gotoh_local(A, B, sub, o, e):
    """Smith-Waterman local alignment score with affine gaps (Gotoh)."""
    nA, nB = len(A), len(B)
    H = np.zeros((nA + 1, nB + 1), dtype=np.int64)
    E = np.full((nA + 1, nB + 1), NEG, dtype=np.int64)
    F = np.full((nA + 1, nB + 1), NEG, dtype=np.int64)
    best = 0
    for i in range(1, nA + 1):
        for j in range(1, nB + 1):
            E[i, j] = max(H[i, j - 1] - o - e, E[i, j - 1] - e)
            F[i, j] = max(H[i - 1, j] - o - e, F[i - 1, j] - e)
            H[i, j] = max(0, H[i - 1, j - 1] + sub[A[i - 1]][B[j - 1]], E[i, j], F[i, j])
            best = max(best, int(H[i, j]))
    return best


def runs_to_steps(ops):
    steps = []
    for w in ops:
        steps += [int(w) & 3] * (int(w) >> 2)
    return steps


def rescore(tc, qc, t_start, q_start, ops, sub, o, e):
    """Score of the alignment written by the run-length ops."""
    t, q, s = t_start, q_start, 0
    for w in ops:
        n, op = int(w) >> 2, int(w) & 3
        if op == 0:
            for u in range(n):
                s += sub[tc[t + u]][qc[q + u]]
            t += n
            q += n
        elif op == 1:
            s -= o + n * e
            q += n
        else:
            s -= o + n * e
            t += n
    return s, t, q


def check_alignment(tc, qc, a, ops, sc):
    """Invariants of one alignment: rescoring equals the score, the ops consume
    exactly its spans, adjacent runs differ, the anchor is an M column, the
    score reaches the gapped threshold, and along each half every H-state point
    stays within Y of the best earlier H-state point of that half."""
    sub, o, e, Y = sc["sub"], sc["gap_open"], sc["gap_extend"], sc["ydrop"]
    s, t, q = rescore(tc, qc, int(a["t_start"]), int(a["q_start"]), ops, sub, o, e)
    assert s == a["score"], (s, a["score"])
    assert t == a["t_end"] and q == a["q_end"]
    assert all((int(ops[x]) & 3) != (int(ops[x + 1]) & 3) for x in range(len(ops) - 1))
    assert a["score"] >= sc["gapped_thresh"]
    # walk the columns, find the anchor, split into halves
    cols = []  # (op, t, q) per step
    t, q = int(a["t_start"]), int(a["q_start"])
    for op in runs_to_steps(ops):
        cols.append((op, t, q))
        if op == 0:
            t, q = t + 1, q + 1
        elif op == 1:
            q += 1
        else:
            t += 1
    idx = [x for x, c in enumerate(cols) if c == (0, int(a["anchor_t"]), int(a["anchor_q"]))]
    assert len(idx) == 1, "anchor column is not an M column of the alignment"
    ax = idx[0]

    def half_ok(steps):
        prefix, best_h = 0, 0
        x = 0
        while x < len(steps):
            op, tt, qq = steps[x]
            if op == 0:
                prefix += sub[tc[tt]][qc[qq]]
                x += 1
            else:
                n = 1
                while x + n < len(steps) and steps[x + n][0] == op:
                    n += 1
                prefix -= o + n * e
                x += n
            assert prefix >= best_h - Y, "Y-drop violated inside the alignment"
            best_h = max(best_h, prefix)

    half_ok(cols[ax + 1:])
    half_ok(cols[:ax][::-1])
    return True
