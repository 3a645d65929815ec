"""GPU checks of the learned cost model through the C ABI: features, BF16
MFMA inference, gradients and Adam training against the CPU oracle
(oracle/mlp.py), the extension log against the oracle's Y-drop halves, the
learned schedule's output against the plain one (bit-exact), and what the
trained network gains over a constant predictor."""
import numpy as np
import pytest

import oracle
from oracle import mlp
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


@pytest.fixture(scope="module")
def case(ctx):
    T, Q = synth.pair_small(n=80_000, divergence=0.15, seed=31, seg_len=4000)
    rng = synth.rng_for(131)
    a = int(rng.integers(0, 40_000))
    Q = [Q[0], T[a:a + 25_000][::-1].copy()]
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    hits = sfe.sfe_seed_hits(ctx, idx, Q)
    hsps = sfe.sfe_ungapped_xdrop(ctx, idx, Q, hits, dict(synth.SCORING))
    log(f"case: {hits.shape[0]} hits, {hsps.shape[0]} HSPs")
    return T, Q, idx, hsps


def init_params(seed):
    """He-uniform initial weights, zero biases (a seeded input, not method arithmetic)."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in mlp.SHAPES:
        lim = np.sqrt(6.0 / i)
        parts.append(rng.uniform(-lim, lim, o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def oracle_features(T, Q, hsps):
    tc, ts = oracle.encode(T)
    out = np.zeros((hsps.shape[0], 16))
    for qid, q in enumerate(Q):
        qc0, qs0 = oracle.encode(q)
        for s in (0, 1):
            qc, qs = (qc0, qs0) if s == 0 else oracle.revcomp(qc0, qs0)
            sel = np.nonzero((hsps["query_id"] == qid) & (hsps["strand"] == s))[0]
            if sel.size == 0:
                continue
            h = np.zeros(sel.size, dtype=[("t0", "i8"), ("q0", "i8"), ("len", "i8"), ("score", "i8")])
            for f in ("t0", "q0", "len", "score"):
                h[f] = hsps[f][sel]
            out[sel] = mlp.features(tc, ts, qc, qs, h, s)
    return out


def test_features_parity(ctx, case):
    T, Q, idx, hsps = case
    log(f"features of {hsps.shape[0]} HSPs")
    got = sfe.sfe_hsp_features(ctx, idx, Q, hsps)
    ref = oracle_features(T, Q, hsps)
    assert got.shape == ref.shape
    err = np.abs(got.astype(np.float64) - ref)
    assert err.max() <= 1e-5, (err.max(), np.unravel_index(err.argmax(), err.shape))


def test_features_of_a_subset_see_only_that_subset(ctx, case):
    T, Q, idx, hsps = case
    sub = hsps[::3].copy()
    got = sfe.sfe_hsp_features(ctx, idx, Q, sub)
    assert np.abs(got.astype(np.float64) - oracle_features(T, Q, sub)).max() <= 1e-5


def test_features_reject_bad_hsps(ctx, case):
    T, Q, idx, hsps = case
    bad = hsps[:2].copy()
    bad["q0"][0] = 10 ** 9
    with pytest.raises(sfe.SfeError):
        sfe.sfe_hsp_features(ctx, idx, Q, bad)


def test_extension_log_targets_match_oracle_halves(ctx, case):
    T, Q, idx, hsps = case
    sub = hsps[: min(80, hsps.shape[0])].copy()
    log(f"extension log of {sub.shape[0]} HSPs")
    f, t = sfe.sfe_extension_log(ctx, idx, Q, sub, dict(synth.SCORING))
    tc, _ = oracle.encode(T)
    sc = dict(synth.SCORING)
    for x in range(sub.shape[0]):
        qc0, qs0 = oracle.encode(Q[int(sub["query_id"][x])])
        qc = qc0 if sub["strand"][x] == 0 else oracle.revcomp(qc0, qs0)[0]
        off = (int(sub["len"][x]) - 1) // 2
        ta, qa = int(sub["t0"][x]) + off, int(sub["q0"][x]) + off
        fb, fi, fj, fc, _ = oracle.ydrop_half(tc[ta + 1:], qc[qa + 1:], sc)
        bb, bi, bj, bc, _ = oracle.ydrop_half(tc[:ta][::-1], qc[:qa][::-1], sc)
        ref = mlp.targets((fc, fi, fj), (bc, bi, bj))
        assert np.allclose(t[x], ref, rtol=0, atol=1e-5), (x, t[x], ref)
    assert np.abs(f.astype(np.float64) - oracle_features(T, Q, sub)).max() <= 1e-5


def test_predict_parity(ctx):
    p = init_params(1)
    p[mlp.NPARAMS - 4:] = [8.0, 6.0, 8.0, 6.0]
    X = np.random.default_rng(2).uniform(0, 1, (1000, 16)).astype(np.float32)
    m = sfe.Model(ctx, p)
    got = m.predict(X)
    ref, _ = mlp.forward(p, X)
    d = np.abs(got - ref)
    log(f"predict: max |d| {d.max():.3g}, median {np.median(d):.3g}")
    assert np.allclose(got, ref, rtol=2e-2, atol=2e-2)
    assert np.median(d) <= 1e-4
    assert np.array_equal(m.params(), p)
    # a ragged count (not a multiple of the 64-row tile)
    got7 = m.predict(X[:7])
    assert np.allclose(got7, got[:7], rtol=0, atol=0)


def test_grad_parity(ctx):
    p = init_params(3)
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 1, (300, 16)).astype(np.float32)
    T = rng.uniform(0, 16, (300, 4)).astype(np.float32)
    m = sfe.Model(ctx, p)
    loss, g = m.grad(X, T)
    rl, rg = mlp.loss_grad(p, X, T)
    rel = np.linalg.norm(g - rg) / np.linalg.norm(rg)
    log(f"grad: loss {loss:.6g} vs {rl:.6g}, relative L2 error {rel:.3g}")
    assert abs(loss - rl) <= 1e-4 * abs(rl)
    assert rel <= 2e-2
    # element by element in every parameter block: |g - g_ref| <= 1e-2 |g_ref| + 1e-3 max|g_ref of the block|.
    # Both sides round activations and back-propagated signals to BF16 at the same points; only the FP32
    # summation order differs, which can move a value across a BF16 rounding boundary (one ulp, 2^-8) for a
    # few of the ~10^5 rounded values.  Such a flip changes one sample's share (1/300 of the mean) of the
    # gradient by 0.4 %, far below 1e-3 of the block's largest element; the relative term covers elements
    # whose value is a sum with little cancellation.
    o = 0
    worst = 0.0
    for rows, cols in mlp.SHAPES:
        for size in (rows * cols, rows):
            blk = slice(o, o + size)
            scale = float(np.abs(rg[blk]).max())
            bound = 1e-2 * np.abs(rg[blk]) + 1e-3 * scale + 1e-9
            dev = np.abs(g[blk] - rg[blk])
            worst = max(worst, float((dev / bound).max()))
            bad = np.nonzero(dev > bound)[0]
            assert bad.size == 0, (o, bad[:8], g[blk][bad[:8]], rg[blk][bad[:8]])
            o += size
    log(f"grad: worst element deviation {worst:.3g} of its bound")


def test_train_parity(ctx):
    p0 = init_params(5)
    rng = np.random.default_rng(6)
    X = rng.uniform(0, 1, (640, 16)).astype(np.float32)
    T = np.stack([8 + 6 * X[:, 0], 5 + 4 * X[:, 1], 8 + 6 * X[:, 2], 5 + 2 * X[:, 3]], 1).astype(np.float32)
    order = np.concatenate([rng.permutation(600) for _ in range(3)]).astype(np.int32)   # ragged last batch
    m = sfe.Model(ctx, p0)
    losses = m.train(X, T, order, batch=64, lr=1e-3)
    p = m.params()
    rp, rl = mlp.train(p0, X, T, order, 64, 1e-3)
    log(f"train: {losses.shape[0]} steps, loss {losses[0]:.4g} -> {losses[-1]:.4g} (oracle {rl[-1]:.4g})")
    assert losses.shape == rl.shape
    assert np.allclose(losses, rl, rtol=2e-2, atol=1e-3)
    assert np.linalg.norm((p - p0) - (rp - p0)) <= 5e-2 * np.linalg.norm(rp - p0)
    # element by element: every parameter's change within 5 % of the oracle's change plus a tenth of one
    # Adam step (lr).  Adam normalises each element's update by its own gradient history, so a gradient
    # element that differs by rounding moves its parameter by at most a fraction of lr per step.
    dev = np.abs((p - p0) - (rp - p0))
    bound = 5e-2 * np.abs(rp - p0) + 1e-4
    log(f"train: worst parameter deviation {float((dev / bound).max()):.3g} of its bound")
    bad = np.nonzero(dev > bound)[0]
    assert bad.size == 0, (bad[:8], (p - p0)[bad[:8]], (rp - p0)[bad[:8]])
    assert losses[-1] < losses[0]


def test_train_rejects_bad_ids(ctx):
    m = sfe.Model(ctx, init_params(7))
    X = np.zeros((10, 16), np.float32)
    T = np.zeros((10, 4), np.float32)
    with pytest.raises(sfe.SfeError):
        m.train(X, T, np.array([0, 10], np.int32), batch=2, lr=1e-3)


def test_learned_schedule_is_bit_exact(ctx, case):
    T, Q, idx, hsps = case
    log("align with the learned persistent schedule")
    m = sfe.Model(ctx, init_params(8))
    a0, o0, s0 = sfe.sfe_align(ctx, idx, Q, dict(synth.SCORING))
    a1, o1, s1 = sfe.sfe_align(ctx, idx, Q, dict(synth.SCORING), schedule=sfe.SFE_SCHED_PERSISTENT, model=m)
    assert np.array_equal(a0, a1)
    assert np.array_equal(o0, o1)
    assert s1["predicted_halves"] == 2 * s1["extensions"] > 0
    assert 0 <= s1["mispredicted_halves"] <= s1["predicted_halves"]
    # adaptive: plain launches for large batches, persistent below the threshold (here: every batch
    # of more than 64 halves goes plain)
    sfe.sfe_ctx_set_tuning(ctx, adaptive_halves=64, persist_waves_per_cu=2)
    try:
        a2, o2, s2 = sfe.sfe_align(ctx, idx, Q, dict(synth.SCORING), schedule=sfe.SFE_SCHED_ADAPTIVE, model=m)
    finally:
        sfe.sfe_ctx_set_tuning(ctx)
    assert np.array_equal(a0, a2) and np.array_equal(o0, o2)
    assert s2["predicted_halves"] == 2 * s2["extensions"]
    # binned: plain launches, predicted-long halves first
    a3, o3, s3 = sfe.sfe_align(ctx, idx, Q, dict(synth.SCORING), schedule=sfe.SFE_SCHED_BINNED, model=m)
    assert np.array_equal(a0, a3) and np.array_equal(o0, o3)
    assert s3["predicted_halves"] == 2 * s3["extensions"]
    ref = oracle.pipeline(T, Q, dict(synth.SCORING))
    assert a1.shape[0] == ref["alns"].shape[0]
    assert np.array_equal(a1["score"].astype(np.int64), ref["alns"]["score"])


def test_trained_model_beats_constant_predictor(ctx):
    """Logs of the plain pipeline on one synthetic pair, a network trained on
    80% of them by the GPU kernels, evaluated on the held-out 20%."""
    T, Q = synth.pair_small(n=400_000, divergence=0.15, seed=41, seg_len=10_000)
    idx = sfe.sfe_build_index(ctx, T, PATTERN, 1, 1)
    hits = sfe.sfe_seed_hits(ctx, idx, Q)
    hsps = sfe.sfe_ungapped_xdrop(ctx, idx, Q, hits, dict(synth.SCORING))
    f, t = sfe.sfe_extension_log(ctx, idx, Q, hsps, dict(synth.SCORING))
    n = f.shape[0]
    log(f"training log: {n} extensions")
    assert n >= 500
    rng = np.random.default_rng(9)
    perm = rng.permutation(n)
    tr, te = perm[: int(0.8 * n)], perm[int(0.8 * n):]
    p0 = init_params(10)
    p0[mlp.NPARAMS - 4:] = t[tr].mean(axis=0)
    m = sfe.Model(ctx, p0)
    order = np.concatenate([rng.permutation(tr) for _ in range(60)]).astype(np.int32)
    m.train(f, t, order, batch=256, lr=2e-3)
    mse = float(np.mean((m.predict(f[te]) - t[te]) ** 2))
    base = float(np.mean((t[tr].mean(axis=0) - t[te]) ** 2))
    log(f"held-out MSE {mse:.4g} vs constant {base:.4g}")
    assert mse < 0.8 * base


def test_train_in_one_graph_equals_eager(ctx):
    """The whole training step sequence recorded in one hipGraph gives the
    same parameters and losses, bit for bit, as eager launches."""
    p0 = init_params(11)
    rng = np.random.default_rng(12)
    X = rng.uniform(0, 1, (500, 16)).astype(np.float32)
    T = rng.uniform(0, 16, (500, 4)).astype(np.float32)
    order = np.concatenate([rng.permutation(500) for _ in range(4)]).astype(np.int32)
    m0 = sfe.Model(ctx, p0)
    l0 = m0.train(X, T, order, batch=100, lr=1e-3)
    sfe.sfe_ctx_set_tuning(ctx, use_graphs=1)
    try:
        m1 = sfe.Model(ctx, p0)
        l1 = m1.train(X, T, order, batch=100, lr=1e-3)
        m2 = sfe.Model(ctx, p0)
        l2 = m2.train(X, T, order, batch=100, lr=1e-3)      # a second capture and launch
    finally:
        sfe.sfe_ctx_set_tuning(ctx, use_graphs=0)
    assert np.array_equal(l0, l1) and np.array_equal(l0, l2)
    assert np.array_equal(m0.params(), m1.params()) and np.array_equal(m0.params(), m2.params())


def test_autotune_picks_a_schedule_and_keeps_results(ctx, case):
    T, Q, idx, hsps = case
    m = sfe.Model(ctx, init_params(13))
    chosen, entries = sfe.sfe_autotune(ctx, idx, Q, dict(synth.SCORING), sample_bases=20_000, model=m)
    log(f"autotune: chosen {chosen}; {len(entries)} candidates")
    # with a model only the schedules that use it compete: persistent and adaptive
    assert len(entries) == 20 and {e["schedule"] for e in entries} == {1, 2, 3}
    assert {e["waves_per_cu"] for e in entries} >= {8, 16}
    assert chosen["max_cells_per_lane"] in (4, 6) and chosen["schedule"] in (1, 2, 3)
    best = min(entries, key=lambda e: e["ms_extend"])
    assert (best["cells_per_lane"], best["schedule"], best["wave_group_cap"]) == (
        chosen["max_cells_per_lane"], chosen["schedule"], chosen["wave_group_cap"])
    try:
        a1, o1, _ = sfe.sfe_align(ctx, idx, Q, dict(synth.SCORING), schedule=chosen["schedule"],
                                  max_cells_per_lane=chosen["max_cells_per_lane"], model=m)
    finally:
        sfe.sfe_ctx_set_tuning(ctx, wave_group_cap=0)
    a0, o0, _ = sfe.sfe_align(ctx, idx, Q, dict(synth.SCORING))
    assert np.array_equal(a0, a1) and np.array_equal(o0, o1)
    # without a model the plain launch competes too
    chosen2, entries2 = sfe.sfe_autotune(ctx, idx, Q, dict(synth.SCORING), sample_bases=20_000)
    sfe.sfe_ctx_set_tuning(ctx, wave_group_cap=0)
    assert len(entries2) == 24 and {e["schedule"] for e in entries2} == {0, 1, 2, 3}


def test_model_save_load_round_trip(ctx, tmp_path):
    """A saved model loads with identical parameters, predictions and Adam state:
    training the loaded copy continues exactly as the original does."""
    rng = np.random.default_rng(17)
    X = rng.uniform(0, 1, (200, 16)).astype(np.float32)
    T = rng.uniform(0, 12, (200, 4)).astype(np.float32)
    order = rng.permutation(200).astype(np.int32)
    m = sfe.Model(ctx, init_params(11))
    m.train(X, T, order, batch=50, lr=1e-3)
    path = str(tmp_path / "cost.sfem")
    m.save(path)
    assert sfe.sfe_model_check_file(path) == sfe.SFE_OK
    m2 = sfe.Model.load(ctx, path)
    assert np.array_equal(m2.params(), m.params())
    assert np.array_equal(m2.predict(X), m.predict(X))
    l1 = m.train(X, T, order, batch=50, lr=1e-3)
    l2 = m2.train(X, T, order, batch=50, lr=1e-3)
    assert np.array_equal(l1, l2)
    assert np.array_equal(m2.params(), m.params())
    # a damaged file is refused through the context as well
    raw = bytearray(open(path, "rb").read())
    raw[40] ^= 1
    bad = tmp_path / "bad.sfem"
    bad.write_bytes(bytes(raw))
    with pytest.raises(sfe.SfeError) as e:
        sfe.Model.load(ctx, str(bad))
    assert e.value.status == sfe.SFE_EINVAL
    m.close()
    m2.close()
