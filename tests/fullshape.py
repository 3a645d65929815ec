"""Properties every committed alignment must have, checked with numpy over
whole alignment sets (test-side only; the column-by-column forms of the same
checks are in refimpl.check_alignment).

Edit operations are run-length words: length << 2 | op, op 0 = M (both
sequences advance), 1 = I (the query advances), 2 = D (the target advances); a
gap run of length L costs gap_open + L * gap_extend.
"""
from __future__ import annotations

import numpy as np


def _runs(alns, ops):
    """Every run of every alignment: (alignment id, length, op), in path order."""
    off = alns["ops_offset" if "ops_offset" in alns.dtype.names else "ops_off"].astype(np.int64)
    ln = alns["ops_len"].astype(np.int64)
    aid = np.repeat(np.arange(ln.shape[0]), ln)
    first = np.cumsum(ln) - ln
    w = ops[off[aid] + (np.arange(aid.shape[0]) - first[aid])].astype(np.int64)
    return aid, first, ln, w >> 2, w & 3


def rescore_all(alns, ops, tc, qc_by_strand, sub, gap_open, gap_extend, chunk=4096):
    """Checks, for every alignment: runs are non-empty and alternate, the ops
    consume exactly [t_start, t_end) x [q_start, q_end) inside the sequences,
    and rescoring them gives the reported score.  Returns the number checked."""
    S = np.asarray(sub, np.int64)
    for c0 in range(0, alns.shape[0], chunk):
        a = alns[c0:c0 + chunk]
        aid, first, ln, n, op = _runs(a, ops)
        assert np.all(ln > 0) and np.all(n > 0) and np.all(op <= 2)
        assert not np.any((op[1:] == op[:-1]) & (aid[1:] == aid[:-1])), "adjacent runs with the same op"
        dt = np.where(op == 1, 0, n)
        dq = np.where(op == 2, 0, n)
        ct, cq = np.cumsum(dt), np.cumsum(dq)
        last = first + ln - 1
        base_t = ct[first] - dt[first]
        base_q = cq[first] - dq[first]
        t_start = a["t_start"].astype(np.int64)
        q_start = a["q_start"].astype(np.int64)
        assert np.array_equal(t_start + ct[last] - base_t, a["t_end"].astype(np.int64))
        assert np.array_equal(q_start + cq[last] - base_q, a["q_end"].astype(np.int64))
        strand = a["strand"].astype(np.int64)
        assert np.all(t_start >= 0) and np.all(a["t_end"].astype(np.int64) <= tc.shape[0])
        qlen = np.array([q.shape[0] for q in qc_by_strand], np.int64)
        assert np.all(q_start >= 0) and np.all(a["q_end"].astype(np.int64) <= qlen[strand])
        # start of each run
        t0 = t_start[aid] + (ct - dt) - base_t[aid]
        q0 = q_start[aid] + (cq - dq) - base_q[aid]
        gap = op != 0
        score = -np.bincount(aid[gap], weights=(gap_open + gap_extend * n[gap]).astype(np.float64),
                             minlength=a.shape[0])
        m = ~gap
        nm = n[m]
        k = np.arange(int(nm.sum())) - np.repeat(np.cumsum(nm) - nm, nm)
        col_t = np.repeat(t0[m], nm) + k
        col_q = np.repeat(q0[m], nm) + k
        col_a = np.repeat(aid[m], nm)
        qall = np.concatenate(qc_by_strand)
        col_q += np.repeat(np.where(strand[aid[m]] == 1, qc_by_strand[0].shape[0], 0), nm)
        score += np.bincount(col_a, weights=S[tc[col_t], qall[col_q]].astype(np.float64), minlength=a.shape[0])
        assert np.array_equal(score.astype(np.int64), a["score"].astype(np.int64)), "rescored score differs"
    return int(alns.shape[0])


def halves_ok(a, ops_a, tc, qc, sub, gap_open, gap_extend, ydrop):
    """One alignment: its anchor is exactly one M column, and along each half
    (the columns after the anchor, and those before it read backwards) every
    H-state point (after an M column or a whole gap run) stays within Y of the
    best earlier point of that half, the half's start (0) included."""
    S = np.asarray(sub, np.int64)
    w = ops_a.astype(np.int64)
    n, op = w >> 2, w & 3
    dt = np.where(op == 1, 0, n)
    dq = np.where(op == 2, 0, n)
    t0 = int(a["t_start"]) + np.cumsum(dt) - dt
    q0 = int(a["q_start"]) + np.cumsum(dq) - dq
    m = op == 0
    nm = n[m]
    k = np.arange(int(nm.sum())) - np.repeat(np.cumsum(nm) - nm, nm)
    col_t = np.repeat(t0[m], nm) + k
    col_q = np.repeat(q0[m], nm) + k
    hit = np.flatnonzero((col_t == int(a["anchor_t"])) & (col_q == int(a["anchor_q"])))
    assert hit.shape[0] == 1, "anchor is not an M column of the alignment"
    # one step per M column or per gap run, in path order
    per_run = np.where(m, n, 1)
    is_col = np.repeat(m, per_run)
    vals = np.empty(is_col.shape[0], np.int64)
    vals[is_col] = S[tc[col_t], qc[col_q]]
    vals[~is_col] = -(gap_open + gap_extend * n[~m])
    ax = int(np.flatnonzero(is_col)[hit[0]])
    for half in (vals[ax + 1:], vals[:ax][::-1]):
        if half.shape[0] == 0:
            continue
        prefix = np.cumsum(half)
        best_before = np.maximum.accumulate(np.concatenate(([0], prefix)))[:-1]
        assert np.all(prefix >= best_before - ydrop), "Y-drop violated inside the alignment"
    return True


def anchors_unique(alns):
    """No two alignments of one (query, strand) share an anchor."""
    key = np.stack([alns["query_id"].astype(np.int64), alns["strand"].astype(np.int64),
                    alns["anchor_t"].astype(np.int64), alns["anchor_q"].astype(np.int64)], axis=1)
    return np.unique(key, axis=0).shape[0] == key.shape[0]
