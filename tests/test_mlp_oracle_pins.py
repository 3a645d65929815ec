"""Pins of the learned-cost-model oracle (oracle/mlp.py) against things other
than itself: torch's bfloat16 cast, torch.nn / autograd / optim.Adam in
float64/float32, central finite differences, exact small-integer networks,
and a hand-worked feature case."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp

HERE = os.path.dirname(os.path.abspath(__file__))


def rand_params(seed, scale=0.3, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(mlp.NPARAMS) * scale).astype(dtype)


def torch_net(p, dtype=torch.float64):
    layers = []
    for li, (W, b) in enumerate(mlp.unpack(np.asarray(p, np.float64))):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).to(dtype)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
        layers.append(lin)
        if li < 3:
            layers.append(torch.nn.ReLU())
    return torch.nn.Sequential(*layers)


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(50000) * 5, rng.standard_normal(1000) * 1e-30,
                        rng.standard_normal(1000) * 1e30]).astype(np.float32)
    # exact halfway cases: ties go to the even neighbour
    ties = np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x00018000, 0x7F7F8000 - 0x10000], dtype=np.uint32)
    x = np.concatenate([x, ties.view(np.float32), np.array([0.0, -0.0, 1.0, -2.5], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16(x).view(np.uint32), ref.view(np.uint32))


def test_parameter_count():
    assert mlp.NPARAMS == 16 * 64 + 64 + 2 * (64 * 64 + 64) + 64 * 4 + 4 == 9668


def test_exact_forward_matches_torch_nn():
    p = rand_params(2)
    X = np.random.default_rng(3).standard_normal((37, 16))
    Y, _ = mlp.forward(p, X, rounded=False, dtype=np.float64)
    ref = torch_net(p)(torch.from_numpy(X)).detach().numpy()
    assert np.allclose(Y, ref, rtol=1e-12, atol=1e-12)


def test_exact_gradient_matches_autograd_and_finite_differences():
    p = rand_params(4)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((23, 16))
    T = rng.standard_normal((23, 4))
    loss, g = mlp.loss_grad(p, X, T, rounded=False, dtype=np.float64)
    net = torch_net(p)
    out = net(torch.from_numpy(X))
    tl = torch.mean((out - torch.from_numpy(T)) ** 2)
    tl.backward()
    ref = np.concatenate([np.concatenate([m.weight.grad.numpy().ravel(), m.bias.grad.numpy()])
                          for m in net if isinstance(m, torch.nn.Linear)])
    assert abs(loss - tl.item()) < 1e-12
    assert np.allclose(g, ref, rtol=1e-10, atol=1e-12)
    # central differences on a spread of parameters (one per layer block and some random)
    idx = [0, 17, 1023, 1050, 1100, 3000, 5200, 7000, 9400, 9500, 9660, 9667]
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_grad(pp, X, T, False, np.float64)[0] - mlp.loss_grad(pm, X, T, False, np.float64)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def exact_case(seed):
    """Sparse power-of-two parameters and 0/1 inputs: the exact float64
    network then often keeps every value on the bf16 grid."""
    rng = np.random.default_rng(seed)
    vals = np.array([-1.0, -0.5, 0.5, 1.0])
    p = np.where(rng.uniform(size=mlp.NPARAMS) < 0.05, vals[rng.integers(0, 4, mlp.NPARAMS)], 0.0)
    X = rng.integers(0, 2, (8, 16)).astype(np.float64)
    T = rng.integers(-4, 5, (8, 4)) / 2.0
    return p, X, T


def test_rounding_is_the_identity_on_exact_values():
    """Where every value of the exact float64 network already lies on the
    bf16 grid, the rounded network (and its gradient) must equal it bit for
    bit: rounding sits only where it should and drops nothing."""
    kept = 0
    for seed in range(200):
        p, X, T = exact_case(seed)
        Ye, acts_e = mlp.forward(p, X, rounded=False, dtype=np.float64)
        le, ge = mlp.loss_grad(p, X, T, rounded=False, dtype=np.float64)
        exact = all(np.array_equal(a, mlp.bf16(a.astype(np.float32)).astype(np.float64)) for a in acts_e)
        exact = exact and np.array_equal(ge, ge.astype(np.float32).astype(np.float64))
        if not exact or not np.any(Ye):
            continue
        kept += 1
        Yr, _ = mlp.forward(p.astype(np.float32), X.astype(np.float32), rounded=True)
        assert np.array_equal(Yr.astype(np.float64), Ye)
        dY = 2 * (Ye - T) / 32
        if not np.array_equal(dY, mlp.bf16(dY.astype(np.float32)).astype(np.float64)):
            continue
        lr, gr = mlp.loss_grad(p.astype(np.float32), X.astype(np.float32), T.astype(np.float32), rounded=True)
        if np.array_equal(ge, mlp.bf16(ge.astype(np.float32)).astype(np.float64)):
            assert np.array_equal(gr.astype(np.float64), ge)
    assert kept >= 5


def test_rounded_path_rounds_activations():
    p = rand_params(6, dtype=np.float32)
    X = np.random.default_rng(7).standard_normal((9, 16)).astype(np.float32)
    _, acts = mlp.forward(p, X, rounded=True)
    for a in acts:
        assert np.array_equal(a.view(np.uint32) & 0xFFFF, np.zeros_like(a.view(np.uint32)))
    Yr, _ = mlp.forward(p, X, rounded=True)
    Ye, _ = mlp.forward(p.astype(np.float64), X.astype(np.float64), rounded=False, dtype=np.float64)
    assert not np.array_equal(Yr.astype(np.float64), Ye)     # rounding really happens
    assert np.allclose(Yr, Ye, rtol=5e-2, atol=5e-2)          # ... and stays small


def test_adam_matches_torch_optim():
    p0 = rand_params(8, dtype=np.float32)
    rng = np.random.default_rng(9)
    grads = [rng.standard_normal(mlp.NPARAMS).astype(np.float32) for _ in range(4)]
    tp = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for s, g in enumerate(grads, 1):
        p, m, v = mlp.adam(p, m, v, g, s, 1e-3)
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
    assert np.allclose(p, tp.detach().numpy(), rtol=1e-6, atol=1e-7)


def test_features_hand_worked():
    g = json.load(open(os.path.join(HERE, "golden", "features_hand.json")))
    tc, ts = oracle.encode(np.frombuffer(g["target"].encode(), np.uint8))
    qc, qs = oracle.encode(np.frombuffer(g["query"].encode(), np.uint8))
    h = np.zeros(len(g["hsps"]), dtype=[("t0", "i8"), ("q0", "i8"), ("len", "i8"), ("score", "i8")])
    for i, r in enumerate(g["hsps"]):
        h[i] = tuple(r)
    f = mlp.features(tc, ts, qc, qs, h, 0)
    assert np.allclose(f, np.array(g["features"]), rtol=0, atol=1e-12)


def windows_case():
    """The hand-worked window case: sequences, HSPs and expected feature values."""
    g = json.load(open(os.path.join(HERE, "golden", "features_windows.json")))
    t = bytearray(b"A" * g["target_len"])
    for pos, ch in g["target_set"].items():
        t[int(pos)] = ord(ch)
    q = bytearray(b"A" * g["query_len"])
    for pos, ch in g["query_set"].items():
        q[int(pos)] = ord(ch)
    return g, np.frombuffer(bytes(t), np.uint8).copy(), np.frombuffer(bytes(q), np.uint8).copy()


def test_features_windows_hand_worked():
    """Every window of the features crossed on both sides: neighbour counts at
    |dt| = 5000 / 5001 and 10000 / 10001, diagonal offsets 64 / 65, GC and
    soft-mask windows of +-1000 bases with marked bases on their first and last
    position, and a window clipped at the sequence start."""
    g, T, Q = windows_case()
    tc, ts = oracle.encode(T)
    qc, qs = oracle.encode(Q)
    h = np.zeros(len(g["hsps"]), dtype=[("t0", "i8"), ("q0", "i8"), ("len", "i8"), ("score", "i8")])
    for i, r in enumerate(g["hsps"]):
        h[i] = tuple(r)
    f = mlp.features(tc, ts, qc, qs, h, 0)
    for name, cols in g["expect"].items():
        row = g["names"].index(name)
        for col, val in cols.items():
            assert abs(f[row, int(col)] - val) <= 1e-12, (name, col, f[row, int(col)], val)


def test_targets_definition():
    t = mlp.targets((7, 2, 3), (0, 0, 0))
    assert np.allclose(t, [3.0, np.log2(6), 0.0, 0.0])


def test_training_beats_constant_predictor():
    """The oracle's own training loop learns a smooth function of the
    features better than the best constant (the mean target)."""
    rng = np.random.default_rng(10)
    X = rng.uniform(0, 1, (1200, 16)).astype(np.float32)
    T = np.stack([8 + 6 * X[:, 0] + 3 * X[:, 1] * X[:, 2], 5 + 4 * X[:, 3],
                  8 + 6 * X[:, 4], 5 + 2 * X[:, 5] + 2 * X[:, 6]], axis=1).astype(np.float32)
    p0 = (rng.standard_normal(mlp.NPARAMS) * 0.1).astype(np.float32)
    tr, te = np.arange(1000), np.arange(1000, 1200)
    order = np.concatenate([rng.permutation(tr) for _ in range(40)])
    p, losses = mlp.train(p0, X, T, order, batch=64, lr=3e-3)
    Yte, _ = mlp.forward(p, X[te])
    mse = np.mean((Yte - T[te]) ** 2)
    base = np.mean((T[tr].mean(axis=0) - T[te]) ** 2)
    assert losses[-1] < losses[0]
    assert mse < 0.25 * base, (mse, base)
