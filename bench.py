"""Benchmark of the seed -> X-drop -> Y-drop pipeline on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic input:
seed hits of the query (both strands) fused with the ungapped X-drop filter,
the HSP set (dedup + order), and the speculative batched gapped Y-drop
extension with traceback and serial commit.  Workloads:

  mid         50 Mbp x 50 Mbp (200 repeat families, 1 % low complexity, 10 + 10
              SVs per Mbp, 25 % divergence); the step also rebuilds the
              position table of the target;
  mid-stress  the same with 3 + 3 SVs per Mbp (homology blocks up to ~630 kbp);
  chrom       1 Gbp target (1000 repeat families, index resident in HBM, built
              once and timed apart) vs a 200 Mbp query (20 large SVs, 35 %
              divergence) streamed as 10 Mbp chunks: step k aligns chunk k;
  chunks      100 Mbp target (the mid recipe) vs --chunks query chunks of
              lognormal length (median 50 kbp, 10 kbp - 2 Mbp), each a target
              segment on a random strand at 10-35 % divergence, all in every
              step: the batched workload;
  segdup      250 Mbp x 250 Mbp at 30 % divergence, the mid target recipe plus
              segmental duplications over 5 % of the target (1-100 kbp copies,
              1-10 % diverged), 10 + 10 SVs per Mbp: the learned-scheduling
              workload;
  small       1 Mbp x 1 Mbp, 15 % divergence.

Inputs are synthetic (seeded), resident in HBM before the timed region.

Two schedules of the gapped stage run on the same steps: plain (one wave per
anchor-half, halves in batch order) and learned: the cost model, trained on
the GPU from extension logs of the first query bases, orders every batch
(halves predicted to be long first, in a plain, binned, persistent or
adaptive launch); the autotuner picks among the schedules that use the
model.  Their outputs must be identical.

Prints one JSON line.  `value` is unique HSPs per second of the whole step
with the faster of the two schedules (`config.schedule` names it); the other
schedule's figures, gapped GCUPS and the other stage rates ride along.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# MI355X: 256 CUs x 64 lanes x 2.4 GHz of int32 VALU lane-ops per second; packed 16-bit
# instructions (v_pk_*_i16/u16) do two lane-ops each
INT32_VALU_PEAK_OPS = 256 * 64 * 2.4e9
INT16X2_VALU_PEAK_OPS = 2 * INT32_VALU_PEAK_OPS
YDROP_OPS_PER_CELL = 12      # E 3, F 3, G 2, H 1, prune 2, best 1
# HBM bytes per extension launch of the mid workload's plain step (rocprofv3 FETCH_SIZE x 2.000 +
# WRITE_SIZE x 1.000, the factors a 1 GiB device copy gives; the traffic summary under profiles/
# holds the commands), valid only for the kernel source the counters were taken on
YDROP_TRAFFIC_BYTES = 70.487e9
YDROP_TRAFFIC_SOURCE_SHA256 = "b9f55cc6e372a45c"
YDROP_TRAFFIC_WORKLOAD = "mid"
XDROP_OPS_PER_COLUMN = 6     # 2 base extracts, index, lookup, add, max / drop test


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name: str, chunks: int = 4096):
    from paper_2606_06811_amd import synth
    if name == "mid":
        T, Q = synth.pair_mid()
        desc = ("50 Mbp target (200 repeat families x 50 copies, 1% soft-masked low complexity) vs 50 Mbp query "
                "(10 inversions + 10 translocations of 20 kbp per Mbp, 25% divergence, 2% indels)")
    elif name == "mid-stress":
        T, Q = synth.pair_mid(sv_per_mbp=3)
        desc = ("50 Mbp target (200 repeat families x 50 copies, 1% soft-masked low complexity) vs 50 Mbp query "
                "(3 inversions + 3 translocations of 20 kbp per Mbp, 25% divergence, 2% indels)")
    elif name == "chrom":
        T, Q = synth.pair_chromosome()
        desc = ("1 Gbp target (1000 repeat families x 50 copies, 1% soft-masked low complexity, index resident in "
                "HBM) vs 200 Mbp query (10 inversions + 10 translocations of 1-5 Mbp, 35% divergence, 2% indels) "
                "streamed in 10 Mbp chunks, one chunk per step")
    elif name == "chunks":
        T, Q = synth.pair_chunks(n_chunks=chunks)
        desc = (f"100 Mbp target (200 repeat families x 50 copies, 1% soft-masked low complexity) vs {chunks} "
                "query chunks of lognormal length (median 50 kbp, 10 kbp-2 Mbp), each a target segment on a "
                "random strand at U(10%, 35%) divergence, 2% indels, all aligned in every step")
    elif name == "segdup":
        T, Q = synth.pair_segdup()
        desc = ("250 Mbp target (200 repeat families x 50 copies, 1% soft-masked low complexity, segmental "
                "duplications over 5% of it: 1-100 kbp copies at 1-10% divergence) vs 250 Mbp query (10 "
                "inversions + 10 translocations of 20 kbp per Mbp, 30% divergence, 2% indels)")
    elif name == "small":
        T, Q = synth.pair_small()
        desc = "1 Mbp target vs 1 Mbp query (3 inversions, 3 translocations of 20 kbp, 15% divergence, 2% indels)"
    else:
        raise SystemExit(f"unknown workload {name}")
    return T, Q, desc


def host_cpu():
    """Model name and logical CPU count of the host (for the baseline's record)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(T, q, sc, what: str):
    """The oracle, single-threaded, on one bounded sample of the workload."""
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    res = oracle.pipeline(T, [q], sc)
    dt = time.perf_counter() - t0
    nh = sum(int(u["hsps"].shape[0]) for u in res["units"])
    model, ncpu = host_cpu()
    info = dict(value=nh / dt, unit="HSPs/s", cores=1, kind="oracle", host_cpu=model, host_logical_cpus=ncpu,
                sample=f"{what}; {nh} unique HSPs, {res['alns'].shape[0]} alignments, {res['ext_cells']} DP "
                       f"cells in {dt:.1f} s on one core")
    return info, res


def sample_parity(ctx, sfe, T, q, sc, ref):
    """The same sample on the GPU (plain schedule): alignments and edit operations must equal the oracle's."""
    import oracle
    import torch
    dev = torch.device("cuda:0")
    idx = sfe.sfe_build_index(ctx, torch.from_numpy(T).to(dev), "1110100110010101111", 1, 1)
    alns, ops, _ = sfe.sfe_align(ctx, idx, [torch.from_numpy(q).to(dev)], sc, cap=1 << 16, ops_cap=1 << 22)
    idx.close()
    ra = ref["alns"]
    ok = alns.shape[0] == ra.shape[0]
    for f in ("query_id", "strand", "t_start", "t_end", "q_start", "q_end", "score", "anchor_t", "anchor_q", "cells"):
        ok = ok and bool(np.array_equal(alns[f].astype(np.int64), ra[f].astype(np.int64)))
    for x in range(alns.shape[0] if ok else 0):
        g = ops[int(alns["ops_offset"][x]):int(alns["ops_offset"][x]) + int(alns["ops_len"][x])]
        ok = ok and bool(np.array_equal(g, oracle.aln_ops(ref, x)))
    return ok, int(alns.shape[0])


def train_cost_model(ctx, sfe, synth, log_fn, T=None, Q=None, train_bp=0, index=None):
    """The learned part: extension logs of every HSP of a training sample, then
    GPU training of the cost model (He-uniform start, seeded).  The sample is
    the first train_bp query bases of the benchmark pair against its whole
    target (the part the timed steps start with), or the 1 Mbp pair when
    train_bp is 0."""
    if train_bp > 0:
        Q = [q[:train_bp] for q in Q]
        what = f"the first {train_bp} query bases of the benchmark pair"
    else:
        T, Q = synth.pair_small()
        what = "the 1 Mbp pair"
    t0 = time.perf_counter()
    idx = index if (index is not None and train_bp > 0) else sfe.sfe_build_index(ctx, T, synth.SEED_PATTERN, 1, 1)
    hits = sfe.sfe_seed_hits(ctx, idx, Q)
    hsps = sfe.sfe_ungapped_xdrop(ctx, idx, Q, hits, dict(synth.SCORING))
    f, t = sfe.sfe_extension_log(ctx, idx, Q, hsps, dict(synth.SCORING))
    if idx is not index:
        idx.close()
    log_fn(f"extension log of {hsps.shape[0]} HSPs in {time.perf_counter() - t0:.1f} s")
    rng = np.random.default_rng(12345)
    parts = []
    for o, i in ((64, 16), (64, 64), (64, 64), (4, 64)):
        lim = np.sqrt(6.0 / i)
        parts += [rng.uniform(-lim, lim, o * i), np.zeros(o)]
    p0 = np.concatenate(parts).astype(np.float32)
    p0[-4:] = t.mean(axis=0)
    model = sfe.Model(ctx, p0)
    n = f.shape[0]
    order = np.concatenate([rng.permutation(n) for _ in range(60)]).astype(np.int32)
    t0 = time.perf_counter()
    losses = model.train(f, t, order, batch=256, lr=2e-3)
    dt = time.perf_counter() - t0
    log_fn(f"cost model trained on {n} extensions of {what}: loss {losses[0]:.3f} -> "
           f"{losses[-1]:.3f} in {len(losses)} steps, {dt:.2f} s")
    return model, dict(source=what, samples=int(n), steps=int(len(losses)), loss_first=float(losses[0]),
                       loss_last=float(losses[-1]), train_s=round(dt, 3))


def truth_sensitivity(alns, ops, origin, qlen):
    """Fraction of the query bases that descend from a target base (origin != -1)
    and lie on an M column pairing them with exactly that base, in some
    committed alignment of the right strand."""
    found = np.zeros(qlen, dtype=bool)
    for x in range(alns.shape[0]):
        a = alns[x]
        runs = ops[int(a["ops_offset"]):int(a["ops_offset"]) + int(a["ops_len"])].astype(np.int64)
        L, op = runs >> 2, runs & 3
        dt = np.where(op != 1, L, 0)
        dq = np.where(op != 2, L, 0)
        t0 = int(a["t_start"]) + np.concatenate([[0], np.cumsum(dt)[:-1]])
        q0 = int(a["q_start"]) + np.concatenate([[0], np.cumsum(dq)[:-1]])
        m = op == 0
        if not m.any():
            continue
        reps = L[m]
        off = np.arange(int(reps.sum())) - np.repeat(np.cumsum(reps) - reps, reps)
        t = np.repeat(t0[m], reps) + off
        q = np.repeat(q0[m], reps) + off
        if int(a["strand"]) == 0:
            ok = origin[q] == t
            found[q[ok]] = True
        else:
            qf = qlen - 1 - q
            ok = origin[qf] == -2 - t
            found[qf[ok]] = True
    hom = origin != -1
    return float(found[hom].sum() / max(int(hom.sum()), 1))


def seed_study(ctx, sfe, synth, sc, log_fn):
    """Spaced seeds on the 1 Mbp pair with its truth map: the paper's 12-of-19
    seed with one transition (step 1) against this project's 14-of-22 seed
    (step 1 and 2): hits, HSPs, alignments, time and sensitivity."""
    import torch
    dev = torch.device("cuda:0")
    out = []
    X, Yf = sfe.SFE_FILTER_XDROP, sfe.SFE_FILTER_YDROP
    cases = [(div, name, pattern, step, flt) for div in (0.15, 0.30)
             for name, pattern, step, flt in (("12-of-19", synth.SEED_PATTERN, 1, X),
                                              ("14-of-22", synth.SEED_PATTERN_14, 1, X),
                                              ("14-of-22", synth.SEED_PATTERN_14, 2, X),
                                              ("12-of-19", synth.SEED_PATTERN, 1, Yf))]
    pairs = {}
    for div, name, pattern, step, flt in cases:
        if div not in pairs:
            pairs[div] = synth.pair_small(divergence=div, truth=True)
        T, Q, origin = pairs[div]
        Td, Qd = torch.from_numpy(T).to(dev), [torch.from_numpy(Q[0]).to(dev)]
        idx = sfe.sfe_build_index(ctx, Td, pattern, 1, step)
        sfe.sfe_align(ctx, idx, Qd, sc, cap=1 << 16, ops_cap=1 << 24, filter=flt)           # warm-up
        t0 = time.perf_counter()
        a, o, st = sfe.sfe_align(ctx, idx, Qd, sc, cap=1 << 16, ops_cap=1 << 24, filter=flt)
        ms = 1e3 * (time.perf_counter() - t0)
        idx.close()
        sens = truth_sensitivity(a, o, origin, Q[0].shape[0])
        out.append(dict(divergence=div, seed=name, pattern=pattern, step=step,
                        filter="ydrop" if flt == Yf else "xdrop", seed_hits=st["seed_hits"], hsps=st["hsps"],
                        alignments=st["committed"], ms_seed_xdrop=round(st["ms_seed_xdrop"], 2),
                        ms_total=round(ms, 2), sensitivity=round(sens, 5)))
        log_fn(f"{div:.2f} divergence, seed {name} step {step}, {'ydrop' if flt == Yf else 'xdrop'} filter: "
               f"{st['seed_hits']} hits, {st['hsps']} HSPs, {st['committed']} alignments, "
               f"{ms:.0f} ms, sensitivity {sens:.4f}")
    return dict(workload="1 Mbp target vs 1 Mbp query (15% and 30% divergence, 3 + 3 SVs), truth map of every "
                         "query base", seeds=out)


def k_sweep(ctx, sfe, synth, sc, Td, Q0d, index, sample_bp, log_fn):
    """Alg. 3's batch size and the two speculation policies on the first
    sample_bp query bases: rounds, extensions, shadow work and time (the
    trade-off of the paper's Sec. 6); every configuration must give the same
    alignments."""
    q = [Q0d[:sample_bp]]
    idx = index or sfe.sfe_build_index(ctx, Td, synth.SEED_PATTERN, 1, 1)
    rows, ref = [], None
    for policy in (sfe.SFE_POLICY_PREFIX, sfe.SFE_POLICY_DEFER):
        for K in (48, 64, 256, 4096, 1 << 20):
            a, o, st = sfe.sfe_align(ctx, idx, q, sc, round_k=K, policy=policy, cap=1 << 18, ops_cap=1 << 24)
            same = True
            if ref is None:
                ref = (a, o)
            else:
                same = bool(np.array_equal(a, ref[0]) and np.array_equal(o, ref[1]))
            needed = st["extensions"] - st["shadow"]
            rows.append(dict(policy="prefix" if policy == sfe.SFE_POLICY_PREFIX else "defer", round_k=K,
                             rounds=st["rounds"], extensions=st["extensions"], shadow=st["shadow"],
                             shadow_fraction=round(st["shadow"] / max(needed, 1), 4), cells=st["cells"],
                             ms_extend=round(st["ms_extend"], 2), ms_total=round(st["ms_total"], 2),
                             identical=same))
            log_fn(f"K sweep {rows[-1]['policy']} K={K}: {st['rounds']} rounds, {st['extensions']} extensions, "
                   f"{st['shadow']} shadow, {st['ms_extend']:.0f} ms extend")
    if idx is not index:
        idx.close()
    return dict(sample=f"first {sample_bp} query bases vs the full target", rows=rows)


def probe_half(n):
    """One forward half along an n-base pair at 25 % divergence, anchored at
    column 50: its time per antidiagonal on one wave (the latency that sets
    the end of every round)."""
    from paper_2606_06811_amd import sfe, synth
    ctx = sfe.sfe_ctx_create(0)
    rng = synth.rng_for(900 + n)
    t = synth.iid_codes(rng, n)
    q, _ = synth.mutate(rng, t, np.zeros(n, bool), 0.25)
    T, Q = synth.to_ascii(t), [synth.to_ascii(q)]
    idx = sfe.sfe_build_index(ctx, T, synth.SEED_PATTERN, 1, 1)
    h = np.zeros(1, sfe.HSP_DTYPE)
    h[0] = (50, 50, 1, 0, 0, 0, (0, 0, 0))
    best = None
    for _ in range(3):
        t0 = time.perf_counter()
        a, o = sfe.sfe_gapped_ydrop(ctx, idx, Q, h, dict(synth.SCORING))
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    k = int(a["t_end"][0] - a["t_start"][0] + a["q_end"][0] - a["q_start"][0])
    print(json.dumps(dict(probe="one gapped half", bases=n, antidiagonals=k, cells=int(a["cells"][0]),
                          score=int(a["score"][0]), ms=round(1e3 * best, 2),
                          us_per_antidiagonal=round(1e6 * best / max(k, 1), 4))), flush=True)
    idx.close()
    ctx.close()


def kernel_sources_digest():
    """Digest of the extension kernel's source and every header it includes (the
    stored HBM traffic figure is valid only for exactly these files)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2606_06811_amd", "csrc")
    h = hashlib.sha256()
    for f in ("k_fused.hip", "ydrop_common.h", "sfe_internal.h", "sfe_kernels.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    with open(os.path.join(ROOT, "include", "sfe.h"), "rb") as fh:
        h.update(b"sfe.h\0" + fh.read())
    return h.hexdigest()


def length_histogram(alns):
    """Committed alignments by target span, in powers of two (bin b: [2^b, 2^(b+1)) bases)."""
    span = (alns["t_end"].astype(np.int64) - alns["t_start"].astype(np.int64)).clip(min=1)
    b = np.floor(np.log2(span)).astype(np.int64)
    return {f"2^{int(k)}": int(v) for k, v in zip(*np.unique(b, return_counts=True))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mid", choices=["mid", "mid-stress", "chrom", "chunks", "segdup", "small"])
    ap.add_argument("--chunks", type=int, default=4096, help="query chunks of the chunks workload")
    ap.add_argument("--round-k", type=int, default=0)
    ap.add_argument("--schedule", default="both", choices=["plain", "learned", "both"],
                    help="both: time the plain schedule and the learned one (the model orders every batch)")
    ap.add_argument("--cpl", type=int, default=0, help="rows per lane of the first band window (0: default)")
    ap.add_argument("--near-band", type=int, default=0, help="deferral nearness band (0: default, <0: off)")
    ap.add_argument("--policy", type=int, default=0, help="0 DEFER, 1 PREFIX (Alg. 3 as printed)")
    ap.add_argument("--tune-bp", type=int, default=-1,
                    help="query bases the autotuner samples for the learned schedule (0: no tuning; -1: default)")
    ap.add_argument("--train-bp", type=int, default=-1,
                    help="query bases whose HSP extensions train the cost model (-1: default)")
    ap.add_argument("--cpu-sample-bp", type=int, default=30_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graphs", action="store_true",
                    help="run the first launch of every batch as a replay of a recorded graph")
    ap.add_argument("--no-studies", action="store_true", help="skip the seed study and the K sweep")
    ap.add_argument("--sweep-bp", type=int, default=1_000_000, help="query bases of the K sweep")
    ap.add_argument("--probe-half", type=int, default=0,
                    help="instead of the benchmark: time one gapped half along an N-base pair at 25%% "
                         "divergence (the per-antidiagonal latency of one wave)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (queries would shard by unit)",
              file=sys.stderr)
        raise SystemExit(2)
    if args.probe_half > 0:
        probe_half(args.probe_half)
        return
    chrom = args.workload == "chrom"
    if args.tune_bp < 0:
        args.tune_bp = 200_000 if chrom else 1_000_000
    if args.train_bp < 0:
        args.train_bp = 200_000 if chrom else 2_000_000

    import torch
    from paper_2606_06811_amd import sfe, synth

    t0 = time.time()
    T, Q, desc = make_workload(args.workload, args.chunks)
    log(f"workload generated in {time.time() - t0:.1f} s: target {T.shape[0]} bp, {len(Q)} queries, "
        f"{sum(q.shape[0] for q in Q)} bp")
    sc = dict(synth.SCORING)
    dev = torch.device("cuda:0")
    Td = torch.from_numpy(T).to(dev)
    Qd = [torch.from_numpy(q).to(dev) for q in Q]
    stream = torch.cuda.current_stream(dev)
    ctx = sfe.sfe_ctx_create(0, stream.cuda_stream)
    torch.cuda.synchronize()

    resident = None
    index_ms = None
    if chrom:
        # the target's position table stays resident; its build is timed apart from the steps
        t0 = time.perf_counter()
        resident = sfe.sfe_build_index(ctx, Td, synth.SEED_PATTERN, 1, 1)
        torch.cuda.synchronize()
        index_ms = 1e3 * (time.perf_counter() - t0)
        log(f"position table of the {T.shape[0]} bp target built in {index_ms:.0f} ms")

    model, train_info, tune_info = None, None, None
    tuned = dict(max_cells_per_lane=args.cpl, schedule=sfe.SFE_SCHED_BINNED, wave_group_cap=0,
                 persist_waves_per_cu=0)
    # training and tuning sample: the first query (its first train_bp / tune_bp bases), or as many
    # leading chunks as hold train_bp bases
    sample_q = Qd[:1]
    if args.workload == "chunks":
        k, tot = 0, 0
        while k < len(Qd) and tot < args.train_bp:
            tot += Qd[k].shape[0]
            k += 1
        sample_q = Qd[:max(k, 1)]
    if args.schedule in ("learned", "both"):
        model, train_info = train_cost_model(ctx, sfe, synth, log, Td, sample_q, args.train_bp, resident)
        if args.tune_bp > 0:
            # autotuner over the schedules that use the model, on the first tune_bp bases of the first query
            t0 = time.perf_counter()
            idx = resident or sfe.sfe_build_index(ctx, Td, synth.SEED_PATTERN, 1, 1)
            tuned, entries = sfe.sfe_autotune(ctx, idx, sample_q, sc, sample_bases=args.tune_bp, model=model,
                                              round_k=args.round_k, policy=args.policy)
            if idx is not resident:
                idx.close()
            tune_info = dict(sample_bases=args.tune_bp, chosen=tuned, seconds=round(time.perf_counter() - t0, 2),
                             candidates=entries)
            log(f"autotune on {args.tune_bp} query bases: {tuned} in {tune_info['seconds']} s")

    sched_name = {sfe.SFE_SCHED_PLAIN: "plain", sfe.SFE_SCHED_PERSISTENT: "persistent",
                  sfe.SFE_SCHED_ADAPTIVE: "adaptive", sfe.SFE_SCHED_BINNED: "binned"}
    peak_used = [0]

    def step(kind, k):
        q = [Qd[k % len(Qd)]] if chrom else Qd
        idx = resident or sfe.sfe_build_index(ctx, Td, synth.SEED_PATTERN, 1, 1)
        # output capacities large enough that the call never has to be repeated for a larger buffer
        big = args.workload in ("chunks", "segdup", "chrom")
        common = dict(round_k=args.round_k, cap=1 << (23 if big else 21), ops_cap=1 << (29 if big else 26),
                      near_band=args.near_band, policy=args.policy)
        if kind == "plain":
            sfe.sfe_ctx_set_tuning(ctx, wave_group_cap=0, use_graphs=int(args.graphs))
            out = sfe.sfe_align(ctx, idx, q, sc, schedule=sfe.SFE_SCHED_PLAIN, max_cells_per_lane=args.cpl,
                                **common)
        else:
            sfe.sfe_ctx_set_tuning(ctx, wave_group_cap=tuned["wave_group_cap"], use_graphs=int(args.graphs),
                                   persist_waves_per_cu=tuned.get("persist_waves_per_cu", 0))
            out = sfe.sfe_align(ctx, idx, q, sc, schedule=tuned["schedule"], model=model,
                                max_cells_per_lane=tuned["max_cells_per_lane"], **common)
        if idx is not resident:
            idx.close()
        free, total = torch.cuda.mem_get_info(dev)
        peak_used[0] = max(peak_used[0], total - free)
        return out

    def run(kind):
        for w in range(args.warmup):
            a, o, s = step(kind, args.steps + w)
            log(f"[{kind}] warmup {w}: {s['hsps']} HSPs, {s['committed']} alignments, {s['rounds']} rounds, "
                f"{s['ms_total']:.0f} ms")
        torch.cuda.synchronize()
        stats, outs = [], []
        t_start = time.perf_counter()
        for k in range(args.steps):
            a, o, s = step(kind, k)
            stats.append(s)
            outs.append((a, o))
            log(f"[{kind}] step {k}: {s['ms_total']:.0f} ms in align (seed+xdrop {s['ms_seed_xdrop']:.0f}, "
                f"hsp set {s['ms_hsp_set']:.0f}, predict {s['ms_predict']:.0f}, extend {s['ms_extend']:.0f}; "
                f"{s['rounds']} rounds, {s['ydrop_launches']} extension launches, "
                f"{s['graph_launches']} graph replays)")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        return dict(ms_step=1e3 * elapsed / args.steps, stats=stats, outs=outs)

    kinds = ["plain", "learned"] if args.schedule == "both" else [args.schedule]
    res = {k: run(k) for k in kinds}
    bit_exact = None
    if len(kinds) == 2:
        bit_exact = all(np.array_equal(a1, a2) and np.array_equal(o1, o2)
                        for (a1, o1), (a2, o2) in zip(res["plain"]["outs"], res["learned"]["outs"]))
    head_kind = min(kinds, key=lambda k: res[k]["ms_step"])
    head = res[head_kind]
    stats = head["stats"]
    ms_step = head["ms_step"]
    hsps = sum(x["hsps"] for x in stats) / len(stats)
    hsps_per_s = hsps / (ms_step / 1e3)

    # dominant kernel: gapped extension (VALU bound; packed int16 when every launch took the
    # 16-bit kernel); live HIP-event timing
    yd_ms = sum(x["ms_ydrop_kernel"] for x in stats)
    yd_cells = sum(x["ydrop_kernel_cells"] for x in stats)
    yd_launches = sum(x["ydrop_launches"] for x in stats)
    sx_ms = sum(x["ms_seed_xdrop_kernel"] for x in stats)
    sx_cols = sum(x["xdrop_columns"] for x in stats)
    yd_ops_s = YDROP_OPS_PER_CELL * yd_cells / (yd_ms / 1e3) if yd_ms > 0 else 0.0
    sx_ops_s = XDROP_OPS_PER_COLUMN * sx_cols / (sx_ms / 1e3) if sx_ms > 0 else 0.0
    dominant = "ydrop" if yd_ms >= sx_ms else "seed_xdrop"
    narrow = all(x["narrow_launches"] == x["ydrop_launches"] for x in stats)
    ext_type = "int16" if narrow else "int32"
    if dominant == "ydrop":
        achieved = yd_ops_s / 1e12
        kname = "k_ydrop_fused16" if narrow else "k_ydrop_fused"
        note = (f"{kname} (extension + traceback): {YDROP_OPS_PER_CELL} {ext_type} ops per DP cell x "
                f"{yd_cells / max(yd_launches, 1):.3g} cells per launch / {yd_ms / max(yd_launches, 1):.3f} ms "
                f"average launch ({yd_launches} launches)")
    else:
        achieved = sx_ops_s / 1e12
        note = (f"k_seed_xdrop: {XDROP_OPS_PER_COLUMN} int32 ops per scanned column x "
                f"{sx_cols / max(len(stats), 1):.3g} columns per launch / {sx_ms / max(len(stats), 1):.3f} ms")
    packed = dominant == "ydrop" and narrow
    peak = (INT16X2_VALU_PEAK_OPS if packed else INT32_VALU_PEAK_OPS) / 1e12
    unit = "Tops/s (int16 lane-ops, two per packed instruction)" if packed else "Tops/s (int32 lane-ops)"
    traffic = None
    if (dominant == "ydrop" and narrow and args.workload == YDROP_TRAFFIC_WORKLOAD
            and kernel_sources_digest().startswith(YDROP_TRAFFIC_SOURCE_SHA256)):
        traffic = YDROP_TRAFFIC_BYTES
    roofline = dict(bound="alu", achieved=round(achieved, 4), peak=round(peak, 2), unit=unit,
                    frac=round(achieved / peak, 5), traffic=traffic, kernel=dominant, note=note)

    seeds, sweep = None, None
    if not args.no_studies:
        sfe.sfe_ctx_set_tuning(ctx)
        seeds = seed_study(ctx, sfe, synth, sc, log)
        sweep = k_sweep(ctx, sfe, synth, sc, Td, Qd[0], resident, args.sweep_bp, log)

    cpu, parity_ok = None, None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        if chrom:
            # the oracle's position table of the whole 1 Gbp target would take minutes to sort:
            # the sample is the first query bases of chunk 0 against the 20 Mbp of target it derives from
            Ts, qs = T[:20_000_000], Q[0][:args.cpu_sample_bp].copy()
            what = (f"first {args.cpu_sample_bp} bases of query chunk 0 (both strands) vs the first 20 Mbp of "
                    f"the target")
        else:
            Ts, qs = T, Q[0][:args.cpu_sample_bp].copy()
            what = f"first {args.cpu_sample_bp} query bases (both strands) vs the full target"
        cpu, ref = cpu_baseline(Ts, qs, sc, what)
        parity_ok, n_par = sample_parity(ctx, sfe, Ts, qs, sc, ref)
        log(f"cpu baseline {cpu['value']:.2f} HSPs/s; the GPU on the same sample: "
            f"{'identical' if parity_ok else 'DIFFERENT'} ({n_par} alignments)")

    def summary(k):
        r = res[k]
        xs = r["stats"]
        pred = sum(x["predicted_halves"] for x in xs)
        mis = sum(x["mispredicted_halves"] for x in xs)
        return dict(ms_per_step=round(r["ms_step"], 2),
                    hsps_per_s=round(sum(x["hsps"] for x in xs) / len(xs) / (r["ms_step"] / 1e3), 2),
                    alignments_per_s=round(sum(x["committed"] for x in xs) / len(xs) / (r["ms_step"] / 1e3), 2),
                    ms_extend=round(sum(x["ms_extend"] for x in xs) / len(xs), 2),
                    ms_ydrop_kernel=round(sum(x["ms_ydrop_kernel"] for x in xs) / len(xs), 2),
                    predicted_halves=pred, mispredicted_halves=mis,
                    misprediction_rate=round(mis / pred, 4) if pred else None,
                    ms_predict=round(sum(x["ms_predict"] for x in xs) / len(xs), 2),
                    schedule=("plain" if k == "plain" else sched_name[tuned["schedule"]] + " + cost model"))

    s = stats[-1]
    hsps_ms = sum(x["ms_seed_xdrop"] for x in stats)
    line = {
        "metric": "HSPs/s + gapped GCUPS, 1 MI355X; learned-binned vs plain batch, bit-exact",
        "value": round(hsps_per_s, 2),
        "unit": "HSPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ext_type,
        "data": "synthetic",
        "config": {"workload": desc, "schedule": summary(head_kind)["schedule"],
                   "policy": "prefix" if args.policy == 1 else "defer",
                   "recorded_graphs": bool(args.graphs),
                   "round_k": sfe.sfe_align_opts_resolve(round_k=args.round_k, policy=args.policy,
                                                         near_band=args.near_band)["round_k"]},
        "gapped_gcups": round(sum(x["cells"] for x in stats) / (sum(x["ms_extend"] for x in stats) / 1e3) / 1e9, 3),
        "gapped_gcups_kernel": round(yd_cells / (yd_ms / 1e3) / 1e9, 3) if yd_ms > 0 else None,
        "seed_hits_per_s": round(sum(x["seed_hits"] for x in stats) / (hsps_ms / 1e3), 1) if hsps_ms > 0 else None,
        "alignments_per_s": round(sum(x["committed"] for x in stats) / len(stats) / (ms_step / 1e3), 2),
        "schedules": {k: summary(k) for k in kinds},
        "learned_vs_plain": (round(res["plain"]["ms_step"] / res["learned"]["ms_step"], 4)
                             if len(kinds) == 2 else None),
        "bit_exact_learned_vs_plain": bit_exact,
        "parity_sample": parity_ok,
        "cost_model_training": train_info,
        "autotune": tune_info,
        "counts": {k: s[k] for k in ("seed_hits", "hsps_raw", "hsps", "rounds", "extensions", "committed",
                                     "shadow", "cells", "overflow_reruns", "xdrop_columns", "ydrop_launches",
                                     "graph_launches", "graph_records")},
        "stage_ms": {k: round(s[k], 2) for k in ("ms_seed_xdrop", "ms_hsp_set", "ms_extend", "ms_total",
                                                 "ms_ydrop_kernel", "ms_seed_xdrop_kernel", "ms_predict")},
        "region_length_histogram": length_histogram(head["outs"][-1][0]),
        "index_build_ms": round(index_ms, 1) if index_ms is not None else None,
        "peak_hbm_used_bytes": int(peak_used[0]),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "seed_study": seeds,
        "k_sweep": sweep,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
