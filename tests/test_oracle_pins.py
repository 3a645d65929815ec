"""Pins of the CPU oracle against things other than itself.

Each test ties one oracle function to a textbook special case, brute force, a
closed form, a hand-worked example or an invariant (see tests/refimpl.py).
All run on the CPU in seconds.
"""
import json
import os

import numpy as np
import pytest

from paper_2606_06811_amd import synth
from tests import refimpl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PATTERN = synth.SEED_PATTERN
BIG = 1 << 29


def codes_of(orc, s: str):
    return orc.encode(np.frombuffer(s.encode(), np.uint8))


def rand_codes(rng, n):
    return synth.iid_codes(rng, n)


def related_pair(seed, n, d):
    rng = synth.rng_for(seed)
    t = synth.iid_codes(rng, n)
    q, _ = synth.mutate(rng, t, np.zeros(n, bool), d)
    return t, q


# --------------------------------------------------------------------------
# alphabet
# --------------------------------------------------------------------------
def test_encode_hand(orc):
    c, s = codes_of(orc, "ACGTNacgtnRyK")
    assert c.tolist() == [0, 1, 2, 3, 4, 0, 1, 2, 3, 4, 4, 4, 4]
    assert s.tolist() == [0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 0, 1, 0]
    with pytest.raises(ValueError):
        codes_of(orc, "ACGX")


def test_revcomp_hand(orc):
    c, s = codes_of(orc, "AACgtN")
    rc, rs = orc.revcomp(c, s)
    # reverse complement of AACGTN is NACGTT; soft flags travel with their bases
    assert rc.tolist() == [4, 0, 1, 2, 3, 3]
    assert rs.tolist() == [0, 1, 1, 0, 0, 0]


# --------------------------------------------------------------------------
# seeds: brute force over every pair of windows
# --------------------------------------------------------------------------
def test_seed_pattern_golden():
    with open(os.path.join(GOLDEN, "seed_pattern.json")) as f:
        g = json.load(f)
    assert g["pattern"] == PATTERN
    assert len(PATTERN) == g["span"] and PATTERN.count("1") == g["weight"]
    assert refimpl.care_offsets(PATTERN) == g["care_offsets"]


@pytest.mark.parametrize("transitions,step", [(1, 1), (0, 1), (1, 3)])
def test_seed_hits_brute_force(orc, transitions, step):
    rng = synth.rng_for(11)
    t = synth.iid_codes(rng, 1500)
    q, _ = synth.mutate(rng, t[200:1400], np.zeros(1200, bool), 0.08)
    q = np.concatenate([synth.iid_codes(rng, 300), q])
    ts = np.zeros(t.shape[0], np.uint8)
    qs = np.zeros(q.shape[0], np.uint8)
    t = t.copy()
    t[700:705] = 4            # N run in the target
    ts[900:930] = 1           # soft-masked run in the target
    q = q.copy()
    qs[50:60] = 1
    q[1000] = 4
    ht, hq = orc.seed_hits(t, ts, q, qs, PATTERN, transitions, step)
    got = set(zip(ht.tolist(), hq.tolist()))
    want = refimpl.brute_seed_hits(t, ts, q, qs, PATTERN, transitions, step)
    assert len(want) > 100
    assert got == want
    # order: (q, t) ascending, no duplicates
    key = hq.astype(np.int64) * (1 << 32) + ht
    assert np.all(np.diff(key) > 0)


def test_seed_hits_identical_sequences(orc):
    rng = synth.rng_for(5)
    t = synth.iid_codes(rng, 800)
    z = np.zeros(800, np.uint8)
    ht, hq = orc.seed_hits(t, z, t, z, PATTERN, 1, 1)
    diag = set(int(a) for a, b in zip(ht, hq) if a == b)
    assert diag == set(range(800 - 19 + 1))


def test_seed_hits_transition_only(orc):
    # one transition at a care position still hits; a transversion does not
    rng = synth.rng_for(6)
    t = synth.iid_codes(rng, 19)
    z = np.zeros(19, np.uint8)
    q1 = t.copy(); q1[0] ^= 2
    q2 = t.copy(); q2[0] ^= 1
    q3 = t.copy(); q3[3] ^= 1     # offset 3 is a don't-care position of the mask
    q4 = t.copy(); q4[0] ^= 2; q4[1] ^= 2
    assert orc.seed_hits(t, z, q1, z, PATTERN, 1, 1)[0].tolist() == [0]
    assert orc.seed_hits(t, z, q1, z, PATTERN, 0, 1)[0].tolist() == []
    assert orc.seed_hits(t, z, q2, z, PATTERN, 1, 1)[0].tolist() == []
    assert orc.seed_hits(t, z, q3, z, PATTERN, 0, 1)[0].tolist() == [0]
    assert orc.seed_hits(t, z, q4, z, PATTERN, 1, 1)[0].tolist() == []


# --------------------------------------------------------------------------
# X-drop
# --------------------------------------------------------------------------
def test_xdrop_closed_form_unbounded(orc, scoring):
    sc = dict(scoring, xdrop=BIG)
    t, q = related_pair(21, 600, 0.2)
    q = q[:600]
    rng = synth.rng_for(22)
    hits_t = rng.integers(0, 600 - 19, 200)
    hits_q = np.clip(hits_t + rng.integers(-3, 4, 200), 0, q.shape[0] - 19)
    got = orc.xdrop(t, q, hits_t, hits_q, 19, sc)
    for x in range(200):
        t0, q0, ln, s = refimpl.xdrop_closed_form(t, q, int(hits_t[x]), int(hits_q[x]), 19, sc["sub"])
        assert (got["t0"][x], got["q0"][x], got["len"][x], got["score"][x]) == (t0, q0, ln, s)


def test_xdrop_hand_cases(orc, scoring):
    with open(os.path.join(GOLDEN, "xdrop_hand.json")) as f:
        cases = json.load(f)
    for c in cases:
        t, _ = codes_of(orc, c["target"])
        q, _ = codes_of(orc, c["query"])
        h = orc.xdrop(t, q, [c["t"]], [c["q"]], 19, dict(scoring, xdrop=c["xdrop"]))[0]
        assert [int(h["t0"]), int(h["q0"]), int(h["len"]), int(h["score"]), int(h["work"])] == c["expect"], c["name"]


def test_xdrop_single_transversion_lowers_seed_score(orc, scoring):
    # in a window of identical bases, one A->T transversion costs 91 + 123 = 214
    rng = synth.rng_for(31)
    t = synth.iid_codes(rng, 19)
    t[5] = 0
    q = t.copy()
    q[5] = 3
    a = orc.xdrop(t, t, [0], [0], 19, scoring)[0]
    b = orc.xdrop(t, q, [0], [0], 19, scoring)[0]
    assert a["score"] - b["score"] == 214


# --------------------------------------------------------------------------
# Y-drop half
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed,nA,nB,d", [(41, 30, 30, 0.0), (42, 40, 37, 0.15), (43, 25, 45, 0.3),
                                          (44, 50, 50, 0.75), (45, 1, 12, 0.2), (46, 0, 5, 0.0)])
def test_ydrop_unbounded_equals_full_gotoh(orc, scoring, seed, nA, nB, d):
    rng = synth.rng_for(seed)
    A = synth.iid_codes(rng, nA)
    B, _ = synth.mutate(rng, A, np.zeros(nA, bool), d) if d > 0 else (A.copy(), None)
    B = np.concatenate([B, synth.iid_codes(rng, max(0, nB - B.shape[0]))])[:nB] if nA else synth.iid_codes(rng, nB)
    sc = dict(scoring, ydrop=BIG)
    best, i, j, cells, ops = orc.ydrop_half(A, B, sc)
    rb, ri, rj, rops = refimpl.gotoh_extension(A.tolist(), B.tolist(), sc["sub"], sc["gap_open"], sc["gap_extend"])
    assert (best, i, j) == (rb, ri, rj)
    assert ops.tolist() == rops
    # with nothing pruned every cell of the (nA+1) x (nB+1) matrix is computed
    assert cells == (nA + 1) * (nB + 1)


def test_ydrop_identical_sequences(orc, scoring):
    rng = synth.rng_for(51)
    A = synth.iid_codes(rng, 300)
    best, i, j, cells, ops = orc.ydrop_half(A, A, scoring)
    assert best == sum(scoring["sub"][a][a] for a in A.tolist())
    assert (i, j) == (300, 300)
    assert ops.tolist() == [0] * 300


def test_ydrop_three_base_insertion(orc, scoring):
    rng = synth.rng_for(52)
    A = synth.iid_codes(rng, 200)
    ins = np.array([(A[99] + 1) % 4, (A[100] + 2) % 4, (A[99] + 3) % 4], np.uint8)
    B = np.concatenate([A[:100], ins, A[100:]])
    best, i, j, cells, ops = orc.ydrop_half(A, B, scoring)
    assert best == sum(scoring["sub"][a][a] for a in A.tolist()) - (400 + 3 * 30)
    assert (i, j) == (200, 203)
    ops = ops.tolist()
    assert ops.count(1) == 3 and ops.count(2) == 0 and ops.count(0) == 200


def test_ydrop_stops_before_costly_block(orc, scoring):
    rng = synth.rng_for(53)
    A1, A2 = synth.iid_codes(rng, 100), synth.iid_codes(rng, 600)
    blockA = np.zeros(300, np.uint8)          # poly-A against poly-T: every pairing
    blockB = np.full(300, 3, np.uint8)        # inside the block is an A/T transversion
    A = np.concatenate([A1, blockA, A2])
    B = np.concatenate([A1, blockB, A2])
    best, i, j, cells, ops = orc.ydrop_half(A, B, scoring)
    assert best == sum(scoring["sub"][a][a] for a in A1.tolist())
    assert (i, j) == (100, 100)
    # crossing the block costs at least 2 (400 + 300 * 30) = 18800 > Y by any
    # mix of A/T columns and gaps; with Y unbounded the 600 matching columns
    # after it pay for the crossing and the half reaches the corner
    b2, i2, j2, _, _ = orc.ydrop_half(A, B, dict(scoring, ydrop=BIG))
    assert b2 > best and (i2, j2) == (1000, 1000)


def test_ydrop_hand_golden(orc, scoring):
    with open(os.path.join(GOLDEN, "ydrop_hand.json")) as f:
        cases = json.load(f)
    for c in cases:
        A, _ = codes_of(orc, c["A"])
        B, _ = codes_of(orc, c["B"])
        sc = dict(scoring, ydrop=c["ydrop"])
        best, i, j, cells, ops = orc.ydrop_half(A, B, sc)
        assert [best, i, j, cells, "".join("MID"[o] for o in ops)] == c["expect"], c["name"]


# --------------------------------------------------------------------------
# whole extension: max over anchors = Smith-Waterman (Gotoh) optimum
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed,n,d", [(61, 30, 0.2), (62, 36, 0.35), (63, 28, 0.6)])
def test_max_over_anchors_is_smith_waterman(orc, scoring, seed, n, d):
    t, q = related_pair(seed, n, d)
    sc = dict(scoring, ydrop=BIG)
    best = max(int(orc.extend(t, q, ta, qa, sc)[0]["score"]) for ta in range(t.shape[0]) for qa in range(q.shape[0]))
    sw = refimpl.gotoh_local(t.tolist(), q.tolist(), sc["sub"], sc["gap_open"], sc["gap_extend"])
    assert sw > 0
    assert best == sw


def test_extension_invariants(orc, scoring):
    t, q = related_pair(71, 3000, 0.15)
    for ta, qa in [(1500, 1500), (100, 98), (2900, 2890), (0, 0)]:
        a, ops = orc.extend(t, q, ta, qa, dict(scoring, gapped_thresh=-BIG))
        a = a.copy()
        refimpl.check_alignment(t, q, a, ops, dict(scoring, gapped_thresh=-BIG))


# --------------------------------------------------------------------------
# pipeline: invariants, commit semantics, speculative equivalence
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_run(orc, scoring):
    T, Q = synth.pair_small(n=40_000, divergence=0.15, seed=7, seg_len=3_000)
    return T, Q, orc.pipeline(T, Q, scoring)


def test_pipeline_invariants(orc, scoring, small_run):
    T, Q, res = small_run
    tc, _ = orc.encode(T)
    qc0, qs0 = orc.encode(Q[0])
    qrc, _ = orc.revcomp(qc0, qs0)
    assert res["alns"].shape[0] >= 2
    for x, a in enumerate(res["alns"]):
        qc = qc0 if a["strand"] == 0 else qrc
        refimpl.check_alignment(tc, qc, a, orc.aln_ops(res, x), scoring)


def test_commit_never_reuses_an_anchor(orc, scoring, small_run):
    T, Q, res = small_run
    tc, _ = orc.encode(T)
    qc0, qs0 = orc.encode(Q[0])
    for u in res["units"]:
        qc = qc0 if u["strand"] == 0 else orc.revcomp(qc0, qs0)[0]
        alns, ops, _, _ = orc.commit_unit(tc, qc, u["hsps"], scoring, 0)
        covered = set()
        for a in alns:
            assert (int(a["anchor_t"]), int(a["anchor_q"])) not in covered
            t, q = int(a["t_start"]), int(a["q_start"])
            for op in refimpl.runs_to_steps(ops[a["ops_off"]:a["ops_off"] + a["ops_len"]]):
                if op == 0:
                    covered.add((t, q))
                    t, q = t + 1, q + 1
                elif op == 1:
                    q += 1
                else:
                    t += 1


def test_hsp_set_order_and_threshold(orc, scoring, small_run):
    _, _, res = small_run
    for u in res["units"]:
        h = u["hsps"]
        assert np.all(h["score"] >= scoring["hsp_thresh"])
        key = list(zip((-h["score"]).tolist(), h["t0"].tolist(), h["q0"].tolist(), h["len"].tolist()))
        assert key == sorted(key) and len(set(key)) == len(key)


@pytest.fixture(scope="module")
def tiny_run(orc, scoring):
    T, Q = synth.pair_small(n=12_000, divergence=0.15, seed=8, seg_len=1_000)
    return T, Q, orc.pipeline(T, Q, scoring)


@pytest.mark.parametrize("K", [1, 2, 7, 48, 64, 1000, 10 ** 9])
def test_speculative_equals_serial(orc, scoring, tiny_run, K):
    """Alg. 3 with any batch size commits exactly what Alg. 1 commits (Sec. 5)."""
    T, Q, res = tiny_run
    tc, _ = orc.encode(T)
    qc0, qs0 = orc.encode(Q[0])
    for u in res["units"]:
        qc = qc0 if u["strand"] == 0 else orc.revcomp(qc0, qs0)[0]
        a1, o1, n1, _ = orc.commit_unit(tc, qc, u["hsps"], scoring, 0)
        a3, o3, n3, _ = orc.commit_unit(tc, qc, u["hsps"], scoring, K)
        assert np.array_equal(a1, a3)
        assert np.array_equal(o1, o3)
        assert n3 >= n1            # speculation can only add (shadow) work


# --------------------------------------------------------------------------
# the commit walk's pass-over decision, against brute force over M columns
# --------------------------------------------------------------------------
def _m_columns(a, ops):
    """Set of (t, q) M columns of one alignment, walked from its start."""
    cols = set()
    t, q = int(a["t_start"]), int(a["q_start"])
    for op in refimpl.runs_to_steps(ops):
        if op == 0:
            cols.add((t, q))
            t, q = t + 1, q + 1
        elif op == 1:
            q += 1
        else:
            t += 1
    return cols


def _expected_walk(orc, tc, qc, hsps, sc):
    """Alg. 1 with the anchor test done by brute force: a set of every M
    column committed so far.  Extensions come from orc.extend (pinned above
    by Gotoh / Smith-Waterman); only the pass-over decision is recomputed."""
    covered = set()
    commits, n_ext = [], 0
    for h in hsps:
        off = (int(h["len"]) - 1) // 2
        ta, qa = int(h["t0"]) + off, int(h["q0"]) + off
        if (ta, qa) in covered:
            continue
        a, ops = orc.extend(tc, qc, ta, qa, sc)
        n_ext += 1
        if int(a["score"]) >= sc["gapped_thresh"]:
            commits.append((a, ops))
            covered |= _m_columns(a, ops)
    return commits, n_ext


def _boundary_probes(a, ops, limit):
    """One-column HSPs whose anchors sit on and just beside the M runs of an
    alignment: a run's first and last column, the columns one before and one
    after it on the same diagonal, and the first column shifted to each
    neighbouring diagonal."""
    probes = []
    t, q = int(a["t_start"]), int(a["q_start"])
    runs = 0
    for w in ops:
        ln, op = int(w) >> 2, int(w) & 3
        if op == 0:
            if runs < limit:
                for pt, pq in ((t - 1, q - 1), (t, q), (t + ln - 1, q + ln - 1), (t + ln, q + ln),
                               (t + 1, q), (t, q + 1)):
                    probes.append((pt, pq))
            runs += 1
            t, q = t + ln, q + ln
        elif op == 1:
            q += ln
        else:
            t += ln
    return probes


@pytest.mark.parametrize("K", [0, 1, 5])
def test_commit_pass_over_matches_brute_force(orc, scoring, K):
    """Every HSP the walk passes over has its anchor on an M column of an
    earlier commit, and every HSP it extends does not (Alg. 1; Alg. 3 with
    batch size K commits the same).  The HSP list is built so that anchors
    fall exactly on, and one column beside, the ends of committed M runs."""
    t, q = related_pair(81, 2500, 0.12)
    sc = dict(scoring)
    first, fops = orc.extend(t, q, 1200, 1200 + (q.shape[0] - t.shape[0]) // 2, dict(sc, gapped_thresh=-BIG))
    # the walk starts with an HSP on a homologous column (on the first extension's path)
    steps = refimpl.runs_to_steps(fops)
    tt, qq = int(first["t_start"]), int(first["q_start"])
    anchor = None
    for op in steps:
        if op == 0 and tt > 1100 and anchor is None:
            anchor = (tt, qq)
        tt, qq = (tt + 1, qq + 1) if op == 0 else ((tt, qq + 1) if op == 1 else (tt + 1, qq))
    assert anchor is not None
    a0, o0 = orc.extend(t, q, anchor[0], anchor[1], sc)
    assert int(a0["score"]) >= sc["gapped_thresh"]
    probes = [anchor] + [p for p in _boundary_probes(a0, o0, 25)
                         if 0 <= p[0] < t.shape[0] and 0 <= p[1] < q.shape[0]]
    hsps = np.zeros(len(probes), orc.HSP_DTYPE)
    hsps["t0"] = [p[0] for p in probes]
    hsps["q0"] = [p[1] for p in probes]
    hsps["len"] = 1
    hsps["score"] = 5000
    want, want_ext = _expected_walk(orc, t, q, hsps, sc)
    got, gops, n_ext, _ = orc.commit_unit(t, q, hsps, sc, K)
    # some probes are covered and some are not: both branches of the decision are exercised
    assert 1 < len(want) and want_ext < len(probes)
    assert len(got) == len(want)
    for x, (a, ops) in enumerate(want):
        g = got[x]
        for f in ("t_start", "t_end", "q_start", "q_end", "score", "anchor_t", "anchor_q"):
            assert int(g[f]) == int(a[f]), (x, f)
        assert np.array_equal(gops[g["ops_off"]:g["ops_off"] + g["ops_len"]], ops)
    if K <= 0:
        assert n_ext == want_ext
    else:
        assert n_ext >= want_ext


# --------------------------------------------------------------------------
# the two-dimensional filter (Y-drop in place of X-drop)
# --------------------------------------------------------------------------
def test_ydrop_filter_unbounded_is_two_gotoh_halves(orc, scoring):
    """With nothing pruned, the 2-D filter's score of a hit is the anchor
    column's substitution score plus the two free-end Gotoh extensions from
    the middle column of its seed window (an independent full-matrix DP), and
    the HSP it yields spans the seed window."""
    rng = synth.rng_for(71)
    t = synth.iid_codes(rng, 110)
    q, _ = synth.mutate(rng, t, np.zeros(110, bool), 0.08, indel=0.03)
    T, Q = synth.to_ascii(t), synth.to_ascii(q)
    tc, ts = orc.encode(T)
    qc, qs = orc.encode(Q)
    sc = dict(scoring, xdrop=BIG)
    ht, hq = orc.seed_hits(tc, ts, qc, qs, synth.SEED_PATTERN, 1, 1)
    assert ht.shape[0] >= 3
    f = orc.ydrop_filter(tc, qc, ht, hq, 19, sc)
    sub, o, e = sc["sub"], sc["gap_open"], sc["gap_extend"]
    for x in range(ht.shape[0]):
        ta, qa = int(ht[x]) + 9, int(hq[x]) + 9
        fwd = refimpl.gotoh_extension(tc[ta + 1:].tolist(), qc[qa + 1:].tolist(), sub, o, e)[0]
        bwd = refimpl.gotoh_extension(tc[:ta][::-1].tolist(), qc[:qa][::-1].tolist(), sub, o, e)[0]
        assert int(f["score"][x]) == sub[tc[ta]][qc[qa]] + fwd + bwd, x
        assert (int(f["t0"][x]), int(f["q0"][x]), int(f["len"][x])) == (int(ht[x]), int(hq[x]), 19)


def test_ydrop_filter_bridges_an_indel(orc, scoring):
    """A 40-base match, a 2-base deletion, then 40 matching bases: the X-drop
    HSP of a seed on either side stops at the gap, the 2-D filter's score
    crosses it (both blocks minus the gap's cost)."""
    rng = synth.rng_for(72)
    left, right = synth.iid_codes(rng, 40), synth.iid_codes(rng, 40)
    gap = synth.iid_codes(rng, 2)
    t = np.concatenate([left, gap, right])
    q = np.concatenate([left, right])
    T, Q = synth.to_ascii(t), synth.to_ascii(q)
    tc, ts = orc.encode(T)
    qc, qs = orc.encode(Q)
    sub = scoring["sub"]
    ht, hq = orc.seed_hits(tc, ts, qc, qs, synth.SEED_PATTERN, 0, 1)
    onleft = (ht == hq) & (ht + 19 <= 40)
    assert onleft.any()
    x = int(np.nonzero(onleft)[0][0])
    xd = orc.xdrop(tc, qc, ht[x:x + 1], hq[x:x + 1], 19, scoring)[0]
    fd = orc.ydrop_filter(tc, qc, ht[x:x + 1], hq[x:x + 1], 19, scoring)[0]
    block = lambda s: sum(sub[int(c)][int(c)] for c in s)
    assert int(xd["score"]) == block(tc[:40])                      # the ungapped scan stops at the gap
    assert int(fd["score"]) == block(tc[:40]) + block(tc[42:]) - (scoring["gap_open"] + 2 * scoring["gap_extend"])
