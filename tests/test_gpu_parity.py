"""Parity of the HIP path with the CPU oracle, element by element, through the
C ABI.  Integer results must be bit-exact.  Sizes are chosen so the oracle
finishes in seconds while the GPU path still spans many 64-window chunks,
several batches and ragged tails."""
import numpy as np
import pytest

import oracle
from paper_2606_06811_amd import sfe, synth

pytestmark = pytest.mark.gpu

PATTERN = synth.SEED_PATTERN


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    log("creating context on device 0")
    c = sfe.sfe_ctx_create(0)
    yield c
    c.close()


def decorate(seq: np.ndarray, rng, n_runs=3, soft_runs=3):
    """Adds N runs and soft-masked (lower-case) runs to an ASCII sequence."""
    s = seq.copy()
    L = s.shape[0]
    for _ in range(n_runs):
        a = int(rng.integers(0, max(1, L - 40)))
        s[a:a + int(rng.integers(1, 30))] = ord("N")
    for _ in range(soft_runs):
        a = int(rng.integers(0, max(1, L - 200)))
        b = a + int(rng.integers(20, 200))
        seg = s[a:b]
        up = (seg >= ord("A")) & (seg <= ord("Z")) & (seg != ord("N"))
        seg[up] += 32
        s[a:b] = seg
    return s


def make_pair(n=50_000, seed=3, div=0.15, nq=1):
    rng = synth.rng_for(seed + 100)
    T, Q = synth.pair_small(n=n, divergence=div, seed=seed, seg_len=max(1000, n // 20))
    T = decorate(T, rng)
    qs = [decorate(Q[0], rng)]
    for k in range(1, nq):
        a = int(rng.integers(0, n // 2))
        piece = T[a:a + n // 3].copy()
        qs.append(piece[::-1].copy() if k % 2 else piece)
    return T, qs


def oracle_units(T, Q, strands=3):
    tc, ts = oracle.encode(T)
    for qid, q in enumerate(Q):
        qc, qs = oracle.encode(q)
        for s in (0, 1):
            if not (strands >> s) & 1:
                continue
            c, m = (qc, qs) if s == 0 else oracle.revcomp(qc, qs)
            yield qid, s, tc, ts, c, m


# ---------------------------------------------------------------------------
# seeds
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("transitions,step,strands,pattern", [
    (1, 1, 3, PATTERN), (0, 1, 3, PATTERN), (1, 3, 1, PATTERN), (1, 1, 2, PATTERN),
    (1, 1, 3, synth.SEED_PATTERN_14), (1, 2, 3, synth.SEED_PATTERN_14)])
def test_seed_hits_parity(ctx, transitions, step, strands, pattern):
    log(f"seed parity transitions={transitions} step={step} strands={strands} pattern={pattern}")
    T, Q = make_pair(n=40_000, seed=5, nq=2)
    idx = sfe.sfe_build_index(ctx, T, pattern, transitions, step)
    got = sfe.sfe_seed_hits(ctx, idx, Q, strands)
    want = []
    for qid, s, tc, ts, c, m in oracle_units(T, Q, strands):
        t, q = oracle.seed_hits(tc, ts, c, m, pattern, transitions, step)
        w = np.zeros(t.shape[0], sfe.HIT_DTYPE)
        w["t"], w["q"], w["query_id"], w["strand"] = t, q, qid, s
        want.append(w)
    want = np.concatenate(want)
    assert want.shape[0] > (1000 if pattern == PATTERN else 100)
    assert got.shape == want.shape
    for f in ("t", "q", "query_id", "strand"):
        assert np.array_equal(got[f], want[f]), f


def test_seed_hits_edge_sequences(ctx):
    log("seed edge sequences")
    rng = synth.rng_for(9)
    T = synth.to_ascii(synth.iid_codes(rng, 5000))
    Q = [np.zeros(0, np.uint8), T[:10].copy(), np.full(300, ord("N"), np.uint8),
         (T[100:400] + 32).astype(np.uint8),
         T[4981:].copy(), T[:19].copy()]
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    got = sfe.sfe_seed_hits(ctx, idx, Q, 3)
    want = []
    for qid, s, tc, ts, c, m in oracle_units(T, Q):
        t, q = oracle.seed_hits(tc, ts, c, m, PATTERN, 1, 1)
        want += [(int(a), int(b), qid, s) for a, b in zip(t, q)]
    assert [(int(h["t"]), int(h["q"]), int(h["query_id"]), int(h["strand"])) for h in got] == want
    assert any(w[2] == 4 for w in want) and any(w[2] == 5 for w in want)   # windows ending at sequence ends


def test_bad_inputs_return_errors(ctx):
    T = np.frombuffer(b"ACGTX" * 10, np.uint8)
    with pytest.raises(sfe.SfeError) as e:
        sfe.sfe_build_index(ctx, T)
    assert e.value.status == sfe.SFE_EINVAL
    good = np.frombuffer(b"ACGT" * 20, np.uint8)
    with pytest.raises(sfe.SfeError):
        sfe.sfe_build_index(ctx, good, "0110")
    with pytest.raises(sfe.SfeError):
        sfe.sfe_build_index(ctx, good, "1" * 15)
    idx = sfe.sfe_build_index(ctx, good)
    with pytest.raises(sfe.SfeError) as e:
        sfe.sfe_align(ctx, idx, [good], dict(synth.SCORING), schedule=4)
    assert e.value.status == sfe.SFE_EINVAL
    for bad in (dict(persist_waves_per_cu=-1), dict(persist_waves_per_cu=65), dict(adaptive_halves=-2)):
        with pytest.raises(sfe.SfeError):
            sfe.sfe_ctx_set_tuning(ctx, **bad)
    sfe.sfe_ctx_set_tuning(ctx, persist_waves_per_cu=4, adaptive_halves=1000)
    assert sfe.sfe_ctx_get_tuning(ctx)["persist_waves_per_cu"] == 4
    sfe.sfe_ctx_set_tuning(ctx)
    idx.close()


# ---------------------------------------------------------------------------
# X-drop and the HSP set
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def seeded(ctx):
    T, Q = make_pair(n=60_000, seed=7, nq=2)
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    hits = sfe.sfe_seed_hits(ctx, idx, Q, 3)
    return T, Q, idx, hits


def test_xdrop_raw_parity(ctx, seeded):
    log("x-drop raw parity")
    T, Q, idx, hits = seeded
    sc = dict(synth.SCORING)
    got = sfe.sfe_ungapped_xdrop(ctx, idx, Q, hits, sc, raw=True)
    assert got.shape[0] == hits.shape[0]
    for qid, s, tc, ts, c, m in oracle_units(T, Q):
        sel = (hits["query_id"] == qid) & (hits["strand"] == s)
        ref = oracle.xdrop(tc, c, hits["t"][sel], hits["q"][sel], 19, sc)
        g = got[sel]
        for f in ("t0", "q0", "len", "score"):
            assert np.array_equal(g[f].astype(np.int64), ref[f]), f


@pytest.mark.parametrize("scale", [1, 200])
def test_xdrop_raw_parity_scaled(ctx, seeded, scale):
    """Scores scaled by 200 no longer fit int8, so the filter reads its 32-bit
    pair table; both tables give the oracle's segments."""
    log(f"x-drop raw parity, scores x{scale}")
    T, Q, idx, hits = seeded
    sc = dict(synth.SCORING)
    sc["sub"] = [[v * scale for v in row] for row in sc["sub"]]
    sc["xdrop"] *= scale
    got = sfe.sfe_ungapped_xdrop(ctx, idx, Q, hits, sc, raw=True)
    for qid, s, tc, ts, c, m in oracle_units(T, Q):
        sel = (hits["query_id"] == qid) & (hits["strand"] == s)
        ref = oracle.xdrop(tc, c, hits["t"][sel], hits["q"][sel], 19, sc)
        for f in ("t0", "q0", "len", "score"):
            assert np.array_equal(got[sel][f].astype(np.int64), ref[f]), f


@pytest.mark.parametrize("xdrop", [910, 0, 1 << 20])
def test_xdrop_edges(ctx, xdrop):
    """Hits placed at and around both sequence ends and the 16-column block
    boundaries of the scan, on a near-identical pair (scans reach the ends)
    with N runs next to some hits: every segment equals the oracle's."""
    log(f"x-drop edge hits, xdrop={xdrop}")
    rng = synth.rng_for(4242)
    n = 700
    t = synth.iid_codes(rng, n)
    q, _ = synth.mutate(rng, t, np.zeros(n, bool), 0.02, indel=0.0)
    m = min(n, q.shape[0])
    T, Qa = synth.to_ascii(t), synth.to_ascii(q[:m])
    for a in (40, 41, 300):
        T[a:a + 3] = ord("N")
    Qa[500:504] = ord("N")
    T[200:260] += 32            # soft-masked: scored like upper case
    sc = dict(synth.SCORING, xdrop=xdrop)
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    span = len(PATTERN)
    pos = sorted({p for b in (0, 16, 32, 48, 64, 250, 480) for p in (b - 1, b, b + 1, b + 15, b + 17)
                  if 0 <= p} | {m - span - k for k in (0, 1, 2, 15, 16, 17, 33)})
    pos = [p for p in pos if p + span <= m]
    pairs = [(a, a) for a in pos] + [(a, b) for a in pos[::3] for b in pos[1::4]]
    hits = np.zeros(len(pairs), sfe.HIT_DTYPE)
    hits["t"] = [a for a, _ in pairs]
    hits["q"] = [b for _, b in pairs]
    got = sfe.sfe_ungapped_xdrop(ctx, idx, [Qa], hits, sc, raw=True)
    tc, _ = oracle.encode(T)
    qc, _ = oracle.encode(Qa)
    ref = oracle.xdrop(tc, qc, hits["t"], hits["q"], span, sc)
    for f in ("t0", "q0", "len", "score"):
        assert np.array_equal(got[f].astype(np.int64), ref[f]), (f, np.nonzero(got[f].astype(np.int64) != ref[f]))
    idx.close()


@pytest.mark.parametrize("xdrop", [910, 0, 1 << 28])
def test_hsp_set_parity(ctx, seeded, xdrop):
    log(f"hsp set parity xdrop={xdrop}")
    T, Q, idx, hits = seeded
    sc = dict(synth.SCORING, xdrop=xdrop, hsp_thresh=2000)
    got = sfe.sfe_ungapped_xdrop(ctx, idx, Q, hits, sc)
    total = 0
    for qid, s, tc, ts, c, m in oracle_units(T, Q):
        sel = (hits["query_id"] == qid) & (hits["strand"] == s)
        ref = oracle.hsp_set(oracle.xdrop(tc, c, hits["t"][sel], hits["q"][sel], 19, sc), sc["hsp_thresh"])
        g = got[(got["query_id"] == qid) & (got["strand"] == s)]
        assert g.shape[0] == ref.shape[0]
        for f in ("t0", "q0", "len", "score"):
            assert np.array_equal(g[f].astype(np.int64), ref[f]), f
        total += g.shape[0]
    assert total > 20
    # global order: query, score descending, strand, t0, q0, len
    key = list(zip(got["query_id"].tolist(), (-got["score"].astype(np.int64)).tolist(), got["strand"].tolist(),
                   got["t0"].tolist(), got["q0"].tolist(), got["len"].tolist()))
    assert key == sorted(key)


# ---------------------------------------------------------------------------
# gapped extension (pure, speculative)
# ---------------------------------------------------------------------------
def compare_extensions(T, Q, hsps, alns, ops, sc):
    tcodes = oracle.encode(T)[0]
    qcodes = {}
    for x in range(hsps.shape[0]):
        h = hsps[x]
        key = (int(h["query_id"]), int(h["strand"]))
        if key not in qcodes:
            qc, qs = oracle.encode(Q[key[0]])
            qcodes[key] = qc if key[1] == 0 else oracle.revcomp(qc, qs)[0]
        off = (int(h["len"]) - 1) // 2
        ra, rops = oracle.extend(tcodes, qcodes[key], int(h["t0"]) + off, int(h["q0"]) + off, sc)
        a = alns[x]
        got = [int(a[f]) for f in ("t_start", "t_end", "q_start", "q_end", "score", "anchor_t", "anchor_q", "cells")]
        want = [int(ra[f]) for f in ("t_start", "t_end", "q_start", "q_end", "score", "anchor_t", "anchor_q", "cells")]
        assert got == want, (x, got, want)
        passed = int(ra["score"]) >= sc["gapped_thresh"]
        assert bool(a["flags"] & 1) == passed
        if passed:
            g = ops[int(a["ops_offset"]):int(a["ops_offset"]) + int(a["ops_len"])]
            assert np.array_equal(g, rops), x


def test_gapped_ydrop_parity(ctx, seeded):
    log("gapped y-drop parity")
    T, Q, idx, hits = seeded
    sc = dict(synth.SCORING)
    hsps = sfe.sfe_ungapped_xdrop(ctx, idx, Q, hits, sc)
    rng = synth.rng_for(1)
    pick = np.sort(rng.choice(hsps.shape[0], size=min(120, hsps.shape[0]), replace=False))
    sub = hsps[pick]
    alns, ops = sfe.sfe_gapped_ydrop(ctx, idx, Q, sub, sc)
    compare_extensions(T, Q, sub, alns, ops, sc)


@pytest.mark.parametrize("ydrop,gap_open,gap_extend", [(9400, 400, 30), (0, 400, 30), (300, 100, 5),
                                                      (2000, 0, 1), (1 << 20, 400, 30)])
def test_gapped_ydrop_scoring_variants(ctx, ydrop, gap_open, gap_extend):
    """Narrow, pruned-to-nothing and very wide bands (the last two force the
    wider register window and the workgroup kernel)."""
    log(f"y-drop variant Y={ydrop} o={gap_open} e={gap_extend}")
    rng = synth.rng_for(ydrop % 97 + gap_extend)
    n = 2500
    t = synth.iid_codes(rng, n)
    q, _ = synth.mutate(rng, t, np.zeros(n, bool), 0.2)
    T, Qs = synth.to_ascii(t), [synth.to_ascii(q)]
    sc = dict(synth.SCORING, ydrop=ydrop, gap_open=gap_open, gap_extend=gap_extend, gapped_thresh=-(1 << 29))
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    h = np.zeros(6, sfe.HSP_DTYPE)
    for x, (t0, q0) in enumerate([(0, 0), (1200, 1190), (2400, 2380), (50, 60), (1000, 1020), (2480, 2480)]):
        q0 = min(q0, Qs[0].shape[0] - 2)
        h[x] = (t0, q0, 1, 0, 0, 0, (0, 0, 0))
    alns, ops = sfe.sfe_gapped_ydrop(ctx, idx, Qs, h, sc)
    compare_extensions(T, Qs, h, alns, ops, sc)


INT8_EXTREMES = [[127, -128, -1, -128, -128], [-128, 127, -128, 0, -128], [0, -128, 127, -128, -128],
                 [-128, -1, -128, 127, -128], [-128, -128, -128, -128, -128]]
NOT_INT8 = [[200, -114, -31, -123, -100], [-114, 100, -125, -31, -100], [-31, -125, 100, -114, -100],
            [-123, -31, -114, 91, -100], [-100, -100, -100, -100, -100]]
# narrow (16-bit) kernel while ydrop + o + e + 2 max|s| + 512 <= 32767: with o=400, e=300
# and HOXD70 (max |s| 125) the last Y that qualifies is 31305
NARROW_CASES = {
    "hoxd70": (synth.HOXD70, 9400, 400, 30),
    "last_narrow_y": (synth.HOXD70, 31305, 400, 300),
    "first_wide_y": (synth.HOXD70, 31306, 400, 300),
    "int8_extremes": (INT8_EXTREMES, 9400, 400, 30),
    "scores_beyond_int8": (NOT_INT8, 9400, 400, 30),
    "no_gap_open": (synth.HOXD70, 3000, 0, 1),
}


@pytest.mark.parametrize("wide", [0, 1])
@pytest.mark.parametrize("case", sorted(NARROW_CASES))
def test_narrow_and_wide_kernels(ctx, case, wide):
    """The packed 16-bit extension (values relative to the Y-drop threshold)
    and the 32-bit one both give the oracle's ends, scores, cells and edit
    operations, at and just past the range limit of the 16-bit kernel."""
    sub, ydrop, gap_open, gap_extend = NARROW_CASES[case]
    log(f"narrow/wide kernel case {case} wide_scores={wide}")
    rng = synth.rng_for(700 + len(case))
    n = 2500
    t = synth.iid_codes(rng, n)
    q, _ = synth.mutate(rng, t, np.zeros(n, bool), 0.15, indel=0.02)
    T, Qs = synth.to_ascii(t), [synth.to_ascii(q)]
    sc = dict(synth.SCORING, sub=sub, ydrop=ydrop, gap_open=gap_open, gap_extend=gap_extend,
              gapped_thresh=-(1 << 29))
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    m = min(len(T), len(Qs[0]))
    h = np.zeros(5, sfe.HSP_DTYPE)
    for x, a in enumerate([0, 7, m // 3, m // 2, m - 2]):
        h[x] = (a, a, 1, 0, 0, 0, (0, 0, 0))
    sfe.sfe_ctx_set_tuning(ctx, wide_scores=wide)
    try:
        alns, ops = sfe.sfe_gapped_ydrop(ctx, idx, Qs, h, sc)
    finally:
        sfe.sfe_ctx_set_tuning(ctx)
    compare_extensions(T, Qs, h, alns, ops, sc)


# ---------------------------------------------------------------------------
# whole pipeline
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def align_case():
    T, Q = make_pair(n=60_000, seed=13, nq=2)
    ref = oracle.pipeline(T, Q, dict(synth.SCORING))
    return T, Q, ref


def compare_alignments(alns, ops, ref):
    ra = ref["alns"]
    assert alns.shape[0] == ra.shape[0], (alns.shape[0], ra.shape[0])
    for f in ("query_id", "strand", "t_start", "t_end", "q_start", "q_end", "score", "anchor_t", "anchor_q", "cells"):
        assert np.array_equal(alns[f].astype(np.int64), ra[f].astype(np.int64)), f
    for x in range(alns.shape[0]):
        g = ops[int(alns["ops_offset"][x]):int(alns["ops_offset"][x]) + int(alns["ops_len"][x])]
        assert np.array_equal(g, oracle.aln_ops(ref, x)), x


PLAIN, PERSIST, ADAPT = sfe.SFE_SCHED_PLAIN, sfe.SFE_SCHED_PERSISTENT, sfe.SFE_SCHED_ADAPTIVE


@pytest.mark.parametrize("K,cpl,policy,schedule", [
    (1, 0, 1, PLAIN), (7, 0, 1, PLAIN), (64, 0, 1, PLAIN), (1000, 0, 1, PLAIN), (64, 4, 1, PLAIN), (64, 8, 1, PLAIN),
    (1, 0, 0, PLAIN), (3, 0, 0, PLAIN), (0, 0, 0, PLAIN), (0, 4, 0, PLAIN),
    (1, 0, 1, PERSIST), (64, 0, 1, PERSIST), (0, 0, 0, PERSIST), (0, 8, 0, PERSIST),
    (0, 0, 0, ADAPT), (7, 0, 1, ADAPT), (0, 0, 0, sfe.SFE_SCHED_BINNED)])
def test_align_parity(ctx, align_case, K, cpl, policy, schedule):
    log(f"align parity K={K} cells_per_lane={cpl} policy={policy} schedule={schedule}")
    T, Q, ref = align_case
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    alns, ops, st = sfe.sfe_align(ctx, idx, Q, dict(synth.SCORING), round_k=K, max_cells_per_lane=cpl,
                                  policy=policy, schedule=schedule)
    assert alns.shape[0] >= 3
    compare_alignments(alns, ops, ref)
    assert st["committed"] == alns.shape[0]
    assert st["extensions"] >= ref["n_extensions"]
    # columns the ungapped filter scored, over every hit, as the oracle counts them
    assert st["xdrop_columns"] == sum(int(u["raw"]["work"].sum()) for u in ref["units"])


@pytest.fixture(scope="module")
def mid_case():
    """The benchmark's generator at 250 kbp: repeat families, soft-masked
    low-complexity runs, inversions and translocations, 25 % divergence."""
    T, Q = synth.pair_mid(n=250_000, families=20, copies=10, seed=21)
    ref = oracle.pipeline(T, Q, dict(synth.SCORING))
    return T, Q, ref


@pytest.mark.parametrize("K,policy", [(0, 0), (64, 1)])
def test_align_parity_mid_shape(ctx, mid_case, K, policy):
    """The whole pipeline on a scaled-down benchmark pair (several deferral
    rounds, long colinear blocks) equals the oracle's Alg. 1 bit for bit."""
    log(f"align parity on a 250 kbp mid-style pair K={K} policy={policy}")
    T, Q, ref = mid_case
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    alns, ops, st = sfe.sfe_align(ctx, idx, Q, dict(synth.SCORING), round_k=K, policy=policy)
    assert alns.shape[0] >= 100
    compare_alignments(alns, ops, ref)
    assert st["xdrop_columns"] == sum(int(u["raw"]["work"].sum()) for u in ref["units"])
    idx.close()


def test_align_parity_wide_scores(ctx, align_case):
    """The whole pipeline on the 32-bit extension kernel."""
    log("align parity with 32-bit extension")
    T, Q, ref = align_case
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    sfe.sfe_ctx_set_tuning(ctx, wide_scores=1)
    try:
        alns, ops, st = sfe.sfe_align(ctx, idx, Q, dict(synth.SCORING))
    finally:
        sfe.sfe_ctx_set_tuning(ctx)
    compare_alignments(alns, ops, ref)


@pytest.mark.parametrize("policy", [0, 1])
def test_align_parity_wave_groups(ctx, align_case, policy):
    """Long halves restarted on wave groups inside the whole pipeline."""
    log(f"align with wave groups, policy={policy}")
    T, Q, ref = align_case
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    sfe.sfe_ctx_set_tuning(ctx, wave_group_cap=1024)
    try:
        alns, ops, st = sfe.sfe_align(ctx, idx, Q, dict(synth.SCORING), policy=policy)
    finally:
        sfe.sfe_ctx_set_tuning(ctx, wave_group_cap=0)
    compare_alignments(alns, ops, ref)
    assert st["overflow_reruns"] > 0


@pytest.mark.parametrize("K,policy,schedule,arena", [
    (7, 1, PLAIN, 0), (64, 1, PERSIST, 0), (0, 0, PLAIN, 0), (0, 0, sfe.SFE_SCHED_BINNED, 0),
    (16, 1, PERSIST, 1 << 20)])
def test_align_parity_recorded_graphs(align_case, K, policy, schedule, arena):
    """The first launch of every batch run as a replay of a recorded graph
    (device-side counts): the same alignments and edit operations as the
    oracle and as stream launches, over two calls on one context (the second
    replays what the first recorded), with stream work and synchronisation
    between the replays; a small arena adds re-runs and regrowth."""
    log(f"align with recorded graphs K={K} policy={policy} schedule={schedule} arena={arena}")
    T, Q, ref = align_case
    c = sfe.sfe_ctx_create(0)
    try:
        idx = sfe.sfe_build_index(c, T, PATTERN, 1, 1)
        kw = dict(round_k=K, policy=policy, schedule=schedule, arena_bytes=arena)
        eager = sfe.sfe_align(c, idx, Q, dict(synth.SCORING), **kw)
        assert eager[2]["graph_launches"] == 0
        sfe.sfe_ctx_set_tuning(c, use_graphs=1)
        launches = records = 0
        for call in range(2):
            alns, ops, st = sfe.sfe_align(c, idx, Q, dict(synth.SCORING), **kw)
            compare_alignments(alns, ops, ref)
            assert np.array_equal(alns, eager[0]) and np.array_equal(ops, eager[1]), call
            assert st["graph_launches"] >= 1, call
            launches += st["graph_launches"]
            records += st["graph_records"]
        assert launches > records        # replays of an earlier recording happened
        sfe.sfe_ctx_set_tuning(c)
        alns, ops, st = sfe.sfe_align(c, idx, Q, dict(synth.SCORING), **kw)
        assert st["graph_launches"] == 0
        assert np.array_equal(alns, eager[0]) and np.array_equal(ops, eager[1])
        idx.close()
    finally:
        c.close()


@pytest.mark.parametrize("arena,schedule", [(1 << 20, PLAIN), (1 << 20, PERSIST), (3 << 18, PLAIN)])
def test_align_tiny_arena_reruns(align_case, arena, schedule):
    """A small traceback arena (fresh context, so the run arena starts small
    too) forces slice-overflow re-runs and run-arena regrowth; results must
    not change."""
    log(f"align with a {arena}-byte arena, schedule={schedule}")
    T, Q, ref = align_case
    c = sfe.sfe_ctx_create(0)
    try:
        idx = sfe.sfe_build_index(c, T, PATTERN, 1, 1)
        alns, ops, st = sfe.sfe_align(c, idx, Q, dict(synth.SCORING), round_k=0, policy=0, arena_bytes=arena,
                                      schedule=schedule)
        compare_alignments(alns, ops, ref)
        assert st["overflow_reruns"] > 0
        idx.close()
    finally:
        c.close()


@pytest.mark.parametrize("n,div,indel", [(30_000, 0.10, 0.02), (20_000, 0.30, 0.05), (12_000, 0.0, 0.0)])
@pytest.mark.parametrize("cap", [0, 2048])
def test_long_halves_on_wave_groups(ctx, n, div, indel, cap):
    """Halves longer than the one-wave antidiagonal cap restart on a group of
    waves; results must equal the oracle's (score, ends, cells, ops)."""
    log(f"long halves n={n} div={div} wave-group cap {cap}")
    sfe.sfe_ctx_set_tuning(ctx, wave_group_cap=cap)
    rng = synth.rng_for(500 + n)
    t = synth.iid_codes(rng, n)
    q, _ = synth.mutate(rng, t, np.zeros(n, bool), div, indel=indel)
    T, Q = synth.to_ascii(t), [synth.to_ascii(q)]
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    h = np.zeros(3, sfe.HSP_DTYPE)
    m = min(len(T), len(Q[0]))
    for x, (a, L) in enumerate([(200, 1), (m // 2, 1), (m - 300, 1)]):
        h[x] = (a, a, L, 0, 0, 0, (0, 0, 0))
    alns, ops = sfe.sfe_gapped_ydrop(ctx, idx, Q, h, dict(synth.SCORING))
    tc, _ = oracle.encode(T)
    qc, _ = oracle.encode(Q[0])
    off = 0
    for x in range(h.shape[0]):
        a, o = oracle.extend(tc, qc, int(h["t0"][x]), int(h["q0"][x]), dict(synth.SCORING))
        for f in ("t_start", "t_end", "q_start", "q_end", "score", "cells"):
            assert int(alns[f][x]) == int(a[f]), (x, f, int(alns[f][x]), int(a[f]))
        if alns["flags"][x] & sfe.SFE_ALN_PASSED:
            g = ops[int(alns["ops_offset"][x]):int(alns["ops_offset"][x]) + int(alns["ops_len"][x])]
            assert np.array_equal(g, o), x
    sfe.sfe_ctx_set_tuning(ctx, wave_group_cap=0)


# ---------------------------------------------------------------------------
# the int32 score guard
# ---------------------------------------------------------------------------
def test_score_range_errors(ctx):
    """Scores that reach 2^29 stop the call with SFE_ERANGE, in the ungapped
    filter (alone and inside the pipeline) and in the gapped extension: a
    20 kbp sequence aligned to itself at 30000 per matching column passes 2^29
    after ~17,900 columns."""
    rng = synth.rng_for(77)
    S = synth.to_ascii(synth.iid_codes(rng, 20_000))
    sc = dict(synth.SCORING)
    sc["sub"] = [[30000 if a == b and a < 4 else -30000 for b in range(5)] for a in range(5)]
    sc["xdrop"] = 1 << 20
    sc["ydrop"] = 1 << 20
    idx = sfe.sfe_build_index(ctx, S, PATTERN, 1, 1)
    log("score range: sfe_align")
    with pytest.raises(sfe.SfeError) as e:
        sfe.sfe_align(ctx, idx, [S], sc)
    assert e.value.status == sfe.SFE_ERANGE
    log("score range: sfe_ungapped_xdrop")
    hits = np.zeros(1, sfe.HIT_DTYPE)
    hits[0] = (100, 100, 0, 0, (0, 0, 0))
    with pytest.raises(sfe.SfeError) as e:
        sfe.sfe_ungapped_xdrop(ctx, idx, [S], hits, sc, raw=True)
    assert e.value.status == sfe.SFE_ERANGE
    log("score range: sfe_gapped_ydrop")
    h = np.zeros(1, sfe.HSP_DTYPE)
    h[0] = (100, 100, 1, 30000, 0, 0, (0, 0, 0))
    with pytest.raises(sfe.SfeError) as e:
        sfe.sfe_gapped_ydrop(ctx, idx, [S], h, sc)
    assert e.value.status == sfe.SFE_ERANGE
    # the same half with a score that stays below the guard succeeds
    sc["sub"] = [[300 if a == b and a < 4 else -300 for b in range(5)] for a in range(5)]
    sc["ydrop"] = 9400
    alns, ops = sfe.sfe_gapped_ydrop(ctx, idx, [S], h, sc)
    assert int(alns["score"][0]) == 300 * 20_000
    idx.close()


# ---------------------------------------------------------------------------
# the two-dimensional (Y-drop) filter in place of X-drop
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("div", [0.15, 0.30])
def test_align_parity_ydrop_filter(ctx, div):
    log(f"align parity with the 2-D filter, divergence {div}")
    rng = synth.rng_for(610)
    T, Q = synth.pair_small(n=20_000, divergence=div, seed=61, seg_len=1500)
    T = decorate(T, rng)
    Q = [decorate(Q[0], rng)]
    sc = dict(synth.SCORING)
    ref = oracle.pipeline(T, Q, sc, filter="ydrop")
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    alns, ops, st = sfe.sfe_align(ctx, idx, Q, sc, filter=sfe.SFE_FILTER_YDROP)
    assert alns.shape[0] >= 2
    compare_alignments(alns, ops, ref)
    assert st["hsps"] == sum(int(u["hsps"].shape[0]) for u in ref["units"])
    assert st["seed_hits"] == sum(int(u["hits_t"].shape[0]) for u in ref["units"])
    idx.close()
