"""Benchmark of the seed -> X-drop -> Y-drop pipeline on one MI355X.

One step = one pass of the whole hot path over the mid-size workload: build
the position table of a 50 Mbp target (2-bit packing, seed keys, sort),
seed hits of a 50 Mbp query on both strands fused with the ungapped X-drop
filter, the HSP set (dedup + order), and the speculative batched gapped
Y-drop extension with traceback and serial commit.  Inputs are synthetic
(seeded), resident in HBM before the timed region.

Two schedules of the gapped stage are timed on the same step: the plain one
(one wave per anchor-half, halves in batch order) and the learned one: the
cost model is trained first, on the GPU, from extension logs of every HSP of
the first 2 Mbp of the query; the autotuner then times candidate schedules
(rows per lane; plain, persistent or adaptive launch with the model's
longest-first order; wave groups for long halves) on a 1 Mbp sample of the
query and the fastest is used (adaptive when no tuning is asked for).  Both run untimed before the timed steps.  Their outputs must
be identical.

Prints one JSON line.  `value` is unique HSPs per second of the whole step
with the learned schedule; the plain schedule's figures, gapped GCUPS and the
other stage rates ride along.
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
YDROP_TRAFFIC_BYTES = 96.593e9
YDROP_TRAFFIC_SOURCE_SHA256 = "6c6ec07e66aa6b57"
XDROP_OPS_PER_COLUMN = 6     # 2 base extracts, index, lookup, add, max / drop test


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name: str):
    from paper_2606_06811_amd import synth
    if name == "mid":
        T, Q = synth.pair_mid()
        desc = "50 Mbp target (200 repeat families x 50 copies, 1% soft-masked low complexity) vs 50 Mbp query (SVs + 25% divergence, 2% indels)"
    elif name == "small":
        T, Q = synth.pair_small()
        desc = "1 Mbp target vs 1 Mbp query (3 inversions, 3 translocations of 20 kbp, 15% divergence, 2% indels)"
    else:
        raise SystemExit(f"unknown workload {name}")
    return T, Q, desc


def cpu_baseline(T, Q, sc, sample_bp: int):
    """The oracle, single-threaded, on the first sample_bp query bases vs the whole target."""
    import oracle
    oracle.build()
    q = [Q[0][:sample_bp].copy()]
    t0 = time.perf_counter()
    res = oracle.pipeline(T, q, sc)
    dt = time.perf_counter() - t0
    nh = sum(int(u["hsps"].shape[0]) for u in res["units"])
    return dict(value=nh / dt, unit="HSPs/s", cores=1, kind="oracle",
                sample=f"first {sample_bp} query bases (both strands) vs the full target; "
                       f"{nh} unique HSPs, {res['alns'].shape[0]} alignments, {res['ext_cells']} DP cells "
                       f"in {dt:.1f} s")


def train_cost_model(ctx, sfe, synth, log_fn, T=None, Q=None, train_bp=0):
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
    idx = sfe.sfe_build_index(ctx, T, synth.SEED_PATTERN, 1, 1)
    hits = sfe.sfe_seed_hits(ctx, idx, Q)
    hsps = sfe.sfe_ungapped_xdrop(ctx, idx, Q, hits, dict(synth.SCORING))
    f, t = sfe.sfe_extension_log(ctx, idx, Q, hsps, dict(synth.SCORING))
    idx.close()
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mid", choices=["mid", "small"])
    ap.add_argument("--round-k", type=int, default=0)
    ap.add_argument("--schedule", default="both", choices=["plain", "persistent", "adaptive", "learned", "both"],
                    help="both: time the plain schedule and the learned, autotuned one (value = learned)")
    ap.add_argument("--cpl", type=int, default=0, help="rows per lane of the first band window (0: default)")
    ap.add_argument("--near-band", type=int, default=0, help="deferral nearness band (0: default, <0: off)")
    ap.add_argument("--tune-bp", type=int, default=1_000_000,
                    help="query bases the autotuner samples for the learned schedule (0: no tuning)")
    ap.add_argument("--train-bp", type=int, default=2_000_000,
                    help="query bases of the benchmark pair whose HSP extensions train the cost model "
                         "(0: the 1 Mbp pair)")
    ap.add_argument("--cpu-sample-bp", type=int, default=30_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (queries would shard by unit)",
              file=sys.stderr)
        raise SystemExit(2)

    import torch
    from paper_2606_06811_amd import sfe, synth

    t0 = time.time()
    T, Q, desc = make_workload(args.workload)
    log(f"workload generated in {time.time() - t0:.1f} s: target {T.shape[0]} bp, query {Q[0].shape[0]} bp")
    sc = dict(synth.SCORING)
    dev = torch.device("cuda:0")
    Td = torch.from_numpy(T).to(dev)
    Qd = [torch.from_numpy(q).to(dev) for q in Q]
    stream = torch.cuda.current_stream(dev)
    ctx = sfe.sfe_ctx_create(0, stream.cuda_stream)
    torch.cuda.synchronize()

    model, train_info, tune_info = None, None, None
    tuned = dict(max_cells_per_lane=args.cpl, schedule=sfe.SFE_SCHED_ADAPTIVE, wave_group_cap=0)
    if args.schedule in ("learned", "both"):
        model, train_info = train_cost_model(ctx, sfe, synth, log, Td, Qd, args.train_bp)
        if args.tune_bp > 0:
            # autotuner: candidate schedules timed on the first tune_bp query bases (untimed setup)
            t0 = time.perf_counter()
            idx = sfe.sfe_build_index(ctx, Td, synth.SEED_PATTERN, 1, 1)
            tuned, entries = sfe.sfe_autotune(ctx, idx, Qd, sc, sample_bases=args.tune_bp, model=model,
                                              round_k=args.round_k)
            idx.close()
            tune_info = dict(sample_bases=args.tune_bp, chosen=tuned, seconds=round(time.perf_counter() - t0, 2),
                             candidates=entries)
            log(f"autotune on {args.tune_bp} query bases: {tuned} in {tune_info['seconds']} s")

    def step(kind):
        idx = sfe.sfe_build_index(ctx, Td, synth.SEED_PATTERN, 1, 1)
        if kind == "plain":
            sfe.sfe_ctx_set_tuning(ctx, wave_group_cap=0)
            out = sfe.sfe_align(ctx, idx, Qd, sc, round_k=args.round_k, schedule=sfe.SFE_SCHED_PLAIN, cap=1 << 21,
                                ops_cap=1 << 26, max_cells_per_lane=args.cpl, near_band=args.near_band)
        else:
            sfe.sfe_ctx_set_tuning(ctx, wave_group_cap=tuned["wave_group_cap"] if kind == "learned" else 0)
            fixed = sfe.SFE_SCHED_ADAPTIVE if kind == "adaptive" else sfe.SFE_SCHED_PERSISTENT
            out = sfe.sfe_align(ctx, idx, Qd, sc, round_k=args.round_k,
                                schedule=tuned["schedule"] if kind == "learned" else fixed,
                                cap=1 << 21, ops_cap=1 << 26, model=model if kind == "learned" else None,
                                max_cells_per_lane=tuned["max_cells_per_lane"] if kind == "learned" else args.cpl,
                                near_band=args.near_band)
        idx.close()
        return out

    def run(kind):
        for w in range(args.warmup):
            a, o, s = step(kind)
            log(f"[{kind}] warmup {w}: {s['hsps']} HSPs, {s['committed']} alignments, {s['rounds']} rounds, "
                f"{s['ms_total']:.0f} ms")
        torch.cuda.synchronize()
        stats = []
        t_start = time.perf_counter()
        for k in range(args.steps):
            a, o, s = step(kind)
            stats.append(s)
            log(f"[{kind}] step {k}: {s['ms_total']:.0f} ms in align (seed+xdrop {s['ms_seed_xdrop']:.0f}, "
                f"hsp set {s['ms_hsp_set']:.0f}, predict {s['ms_predict']:.0f}, extend {s['ms_extend']:.0f})")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        return dict(ms_step=1e3 * elapsed / args.steps, stats=stats, alns=a, ops=o)

    kinds = ["plain", "learned"] if args.schedule == "both" else [args.schedule]
    res = {k: run(k) for k in kinds}
    head = res[kinds[-1]]
    bit_exact = None
    if len(kinds) == 2:
        bit_exact = bool(np.array_equal(res["plain"]["alns"], res["learned"]["alns"])
                         and np.array_equal(res["plain"]["ops"], res["learned"]["ops"]))
    stats = head["stats"]
    ms_step = head["ms_step"]
    s = stats[-1]
    hsps_per_s = s["hsps"] / (ms_step / 1e3)

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
    if dominant == "ydrop" and narrow and args.workload == "mid":
        import hashlib
        src = os.path.join(ROOT, "paper_2606_06811_amd", "csrc", "k_fused.hip")
        with open(src, "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest().startswith(YDROP_TRAFFIC_SOURCE_SHA256):
                traffic = YDROP_TRAFFIC_BYTES
    roofline = dict(bound="alu", achieved=round(achieved, 4), peak=round(peak, 2), unit=unit,
                    frac=round(achieved / peak, 5), traffic=traffic, kernel=dominant, note=note)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(T, Q, sc, args.cpu_sample_bp)

    def summary(k):
        r = res[k]
        x = r["stats"][-1]
        return dict(ms_per_step=round(r["ms_step"], 2), hsps_per_s=round(x["hsps"] / (r["ms_step"] / 1e3), 2),
                    alignments_per_s=round(x["committed"] / (r["ms_step"] / 1e3), 2),
                    ms_extend=round(x["ms_extend"], 2), ms_ydrop_kernel=round(x["ms_ydrop_kernel"], 2),
                    predicted_halves=x["predicted_halves"], mispredicted_halves=x["mispredicted_halves"],
                    misprediction_rate=(round(x["mispredicted_halves"] / x["predicted_halves"], 4)
                                        if x["predicted_halves"] else None),
                    ms_predict=round(x["ms_predict"], 2))

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
        "config": {"workload": desc, "schedule": kinds[-1], "policy": "defer",
                   "round_k": args.round_k or (1 << 20)},
        "gapped_gcups": round(s["cells"] / (s["ms_extend"] / 1e3) / 1e9, 3) if s["ms_extend"] > 0 else None,
        "gapped_gcups_kernel": round(yd_cells / (yd_ms / 1e3) / 1e9, 3) if yd_ms > 0 else None,
        "seed_hits_per_s": round(s["seed_hits"] / (s["ms_seed_xdrop"] / 1e3), 1) if s["ms_seed_xdrop"] > 0 else None,
        "alignments_per_s": round(s["committed"] / (ms_step / 1e3), 2),
        "schedules": {k: summary(k) for k in kinds},
        "learned_vs_plain": (round(res["plain"]["ms_step"] / res["learned"]["ms_step"], 4)
                             if len(kinds) == 2 else None),
        "bit_exact_learned_vs_plain": bit_exact,
        "cost_model_training": train_info,
        "autotune": tune_info,
        "counts": {k: s[k] for k in ("seed_hits", "hsps_raw", "hsps", "rounds", "extensions", "committed",
                                     "shadow", "cells", "overflow_reruns", "xdrop_columns")},
        "stage_ms": {k: round(s[k], 2) for k in ("ms_seed_xdrop", "ms_hsp_set", "ms_extend", "ms_total",
                                                 "ms_ydrop_kernel", "ms_seed_xdrop_kernel", "ms_predict")},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
