"""The benchmark's default workload at full size (50 Mbp target x 50 Mbp
query, repeat families, soft-masked low-complexity runs, inversions and
translocations, 25 % divergence) on the GPU, in the launch configuration the
benchmark times: plain schedule, default batch policy and band, no recorded
graphs.  The oracle cannot align the whole pair in test time, so

* every alignment of the full run is checked by properties that hold at any
  size (tests/fullshape.py): rescoring its edit operations gives its score and
  end coordinates inside the sequences, runs alternate, anchors are unique per
  strand, scores reach the gapped threshold; a seeded sample of 2,000
  alignments plus the 20 longest also have their anchor on one M column and
  the Y-drop rule along both halves;
* a 10 kbp query sample against the whole 50 Mbp target (the position table
  and every repeat family of the full run) is compared with the oracle
  alignment by alignment and op by op.
"""
import numpy as np
import pytest

import oracle
from paper_2606_06811_amd import sfe, synth
from tests import fullshape

pytestmark = pytest.mark.gpu

SAMPLE_BP = 10_000


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _align(ctx, idx, q, sc, cap, ops_cap):
    sfe.sfe_ctx_set_tuning(ctx, wave_group_cap=0, use_graphs=0)
    return sfe.sfe_align(ctx, idx, q, sc, schedule=sfe.SFE_SCHED_PLAIN, max_cells_per_lane=0, round_k=0,
                         near_band=0, policy=0, cap=cap, ops_cap=ops_cap)


@pytest.fixture(scope="module")
def full():
    import torch
    log("generating the 50 Mbp x 50 Mbp pair")
    T, Q = synth.pair_mid()
    dev = torch.device("cuda:0")
    ctx = sfe.sfe_ctx_create(0)
    log("building the position table on cuda:0")
    idx = sfe.sfe_build_index(ctx, torch.from_numpy(T).to(dev), synth.SEED_PATTERN, 1, 1)
    yield T, Q, ctx, idx, dev
    idx.close()
    ctx.close()


def test_full_run_alignment_properties(full):
    import torch
    T, Q, ctx, idx, dev = full
    sc = dict(synth.SCORING)
    log("aligning the full pair (plain schedule)")
    alns, ops, st = _align(ctx, idx, [torch.from_numpy(Q[0]).to(dev)], sc, 1 << 21, 1 << 26)
    n = alns.shape[0]
    log(f"{n} alignments, {st['rounds']} rounds; checking them")
    assert n > 100_000
    assert np.all(alns["query_id"] == 0)
    assert np.all(alns["score"] >= sc["gapped_thresh"])
    assert fullshape.anchors_unique(alns)
    tc, _ = oracle.encode(T)
    qc0, qs0 = oracle.encode(Q[0])
    qrc, _ = oracle.revcomp(qc0, qs0)
    qcs = [qc0, qrc]
    assert fullshape.rescore_all(alns, ops, tc, qcs, sc["sub"], sc["gap_open"], sc["gap_extend"]) == n
    span = alns["t_end"].astype(np.int64) - alns["t_start"].astype(np.int64)
    pick = set(np.random.default_rng(5).choice(n, 2000, replace=False).tolist())
    pick |= set(np.argsort(span)[-20:].tolist())
    log(f"Y-drop rule along both halves of {len(pick)} alignments (longest {int(span.max())} bases)")
    for x in sorted(pick):
        a = alns[x]
        o = ops[int(a["ops_offset"]):int(a["ops_offset"]) + int(a["ops_len"])]
        fullshape.halves_ok(a, o, tc, qcs[int(a["strand"])], sc["sub"], sc["gap_open"], sc["gap_extend"],
                            sc["ydrop"])


def test_full_target_query_sample_matches_oracle(full):
    import torch
    T, Q, ctx, idx, dev = full
    sc = dict(synth.SCORING)
    q = Q[0][:SAMPLE_BP].copy()
    log(f"oracle: first {SAMPLE_BP} query bases against the full target")
    ref = oracle.pipeline(T, [q], sc)
    alns, ops, _ = _align(ctx, idx, [torch.from_numpy(q).to(dev)], sc, 1 << 16, 1 << 22)
    ra = ref["alns"]
    log(f"{ra.shape[0]} alignments from the oracle, {alns.shape[0]} from the GPU")
    assert ra.shape[0] > 0
    assert alns.shape[0] == ra.shape[0]
    for f in ("query_id", "strand", "t_start", "t_end", "q_start", "q_end", "score", "anchor_t", "anchor_q",
              "cells"):
        assert np.array_equal(alns[f].astype(np.int64), ra[f].astype(np.int64)), f
    for x in range(alns.shape[0]):
        g = ops[int(alns["ops_offset"][x]):int(alns["ops_offset"][x]) + int(alns["ops_len"][x])]
        assert np.array_equal(g, oracle.aln_ops(ref, x)), x
