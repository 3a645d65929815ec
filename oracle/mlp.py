"""CPU oracle of the learned cost model: per-HSP features, the 16-64-64-64-4
MLP (forward, MSE loss, backward) and its Adam update.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may use this module; the product library never does.

The paper motivates the model without defining it: extension sizes cannot be
known before the extension runs (Sec. 8, the cost of an anchor-half is
unpredictable), and better load balancing by sorting work up front is left
as future work (Sec. 9).  So the network, its features and its precision are
readings of this project, stated here as plain definitions:

* parameters, in this order, each row-major (out x in): W1 64x16, b1 64,
  W2 64x64, b2 64, W3 64x64, b3 64, W4 4x64, b4 4 -- 9668 floats (FP32
  master copy);
* forward: every parameter and the input are rounded to BF16
  (round-to-nearest-even); each hidden layer computes Z = X W^T + b with FP32
  accumulation and passes on A = bf16(relu(Z)); the output layer is linear,
  FP32, not rounded;
* loss: mean over the batch and the 4 outputs of (Y - T)^2;
* backward: dY = 2 (Y - T) / (4 B) is rounded to BF16 before it meets a
  product, and so is every back-propagated signal dZ = dA * [A > 0]; weight
  gradients are G^T A_prev and bias gradients column sums of G, FP32; the
  rounding of weights passes the gradient straight through to the master copy;
* Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master weights.

With ``rounded=False`` and float64 the same functions give the exact network,
which the tests pin against finite differences and autograd.
"""
from __future__ import annotations

import numpy as np

NIN, NHID, NOUT = 16, 64, 4
SHAPES = [(NHID, NIN), (NHID, NHID), (NHID, NHID), (NOUT, NHID)]
NPARAMS = sum(o * i + o for o, i in SHAPES)       # 9668


def bf16(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); finite inputs."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def unpack(p: np.ndarray):
    """[(W1, b1), ..., (W4, b4)] as views of the flat parameter vector."""
    out, o = [], 0
    for rows, cols in SHAPES:
        W = p[o:o + rows * cols].reshape(rows, cols)
        o += rows * cols
        b = p[o:o + rows]
        o += rows
        out.append((W, b))
    return out


def forward(p, X, rounded=True, dtype=np.float32):
    """Returns (output Y, activations [X, A1, A2, A3]) of a batch X (B x 16)."""
    r = bf16 if rounded else (lambda a: a)
    layers = unpack(np.asarray(p, dtype=dtype))
    A = r(np.asarray(X, dtype=dtype)).astype(dtype)
    acts = [A]
    for li, (W, b) in enumerate(layers):
        Wr, br = r(W).astype(dtype), r(b).astype(dtype)
        Z = A @ Wr.T + br
        if li == len(layers) - 1:
            return Z, acts
        A = r(np.maximum(Z, 0)).astype(dtype)
        acts.append(A)
    raise AssertionError


def loss_grad(p, X, T, rounded=True, dtype=np.float32):
    """Mean squared error of the batch and its gradient (flat, parameter order)."""
    r = bf16 if rounded else (lambda a: a)
    Y, acts = forward(p, X, rounded, dtype)
    T = np.asarray(T, dtype=dtype)
    B = X.shape[0]
    diff = Y - T
    loss = float(np.mean(diff.astype(np.float64) ** 2))
    layers = unpack(np.asarray(p, dtype=dtype))
    grads = [None] * len(layers)
    G = r(2 * diff / dtype(4 * B)).astype(dtype)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        A_prev = acts[li]
        grads[li] = (G.T @ A_prev, G.sum(axis=0))
        if li == 0:
            break
        dA = G @ r(W).astype(dtype)
        G = r(dA * (A_prev > 0)).astype(dtype)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat.astype(dtype)


def adam(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v), float32."""
    f = np.float32
    m = f(b1) * m + f(1 - b1) * g
    v = f(b2) * v + f(1 - b2) * g * g
    mh = m / f(1 - b1 ** step)
    vh = v / f(1 - b2 ** step)
    p = p - f(lr) * mh / (np.sqrt(vh) + f(eps))
    return p.astype(np.float32), m.astype(np.float32), v.astype(np.float32)


def train(p0, X, T, order, batch, lr):
    """Adam over the batches of `order` (a flat list of sample ids, consumed
    `batch` at a time; a short last batch is used as is).  Returns the final
    parameters and the loss of every batch."""
    p = np.array(p0, dtype=np.float32)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    step = 0
    for s in range(0, len(order), batch):
        ids = np.asarray(order[s:s + batch])
        loss, g = loss_grad(p, X[ids], T[ids])
        step += 1
        p, m, v = adam(p, m, v, g, step, lr)
        losses.append(loss)
    return p, np.array(losses)


# ---------------------------------------------------------------------------
# features of an HSP
# ---------------------------------------------------------------------------
FEATURE_NAMES = [
    "score/4096", "log2(1+len)/16", "identity", "transitions/len", "other mismatches/len",
    "(t0-q0)/n_t", "strand", "ta/n_t", "qa/n_q", "target GC +-1000", "query GC +-1000",
    "log2(1+near-diagonal HSPs +-5000)/8", "log2(1+HSPs +-10000)/8",
    "log2(1+gap to next near-diagonal HSP downstream)/16", "same upstream", "target soft-masked +-1000",
]
NEAR_DIAG, NEAR_T, WIDE_T, GC_W = 64, 5000, 10000, 1000


def _gc(codes, lo, hi):
    """GC fraction of the non-N bases of [lo, hi) (0 if there are none)."""
    lo, hi = max(lo, 0), min(hi, len(codes))
    n = gc = 0
    for p in range(lo, hi):
        if codes[p] < 4:
            n += 1
            gc += codes[p] in (1, 2)
    return gc / n if n else 0.0


def _soft(soft, lo, hi):
    lo, hi = max(lo, 0), min(hi, len(soft))
    return float(np.count_nonzero(soft[lo:hi])) / (hi - lo) if hi > lo else 0.0


def features(tc, tsoft, qc, qsoft, hsps, strand):
    """16 features per HSP of one (query, strand) unit.  tc/qc are codes
    (0-3, 4 = N) of the target and of the strand's query, tsoft/qsoft their
    soft-mask flags; hsps has fields t0, q0, len, score (the unit's unique
    HSPs: the neighbourhood features count within this set).  float64."""
    n = len(hsps)
    nt, nq = len(tc), len(qc)
    out = np.zeros((n, 16), dtype=np.float64)
    ta = [int(h["t0"]) + (int(h["len"]) - 1) // 2 for h in hsps]
    qa = [int(h["q0"]) + (int(h["len"]) - 1) // 2 for h in hsps]
    dg = [ta[x] - qa[x] for x in range(n)]
    for x, h in enumerate(hsps):
        t0, q0, L, sc = int(h["t0"]), int(h["q0"]), int(h["len"]), int(h["score"])
        match = ts = tv = 0
        for u in range(L):
            a, b = int(tc[t0 + u]), int(qc[q0 + u])
            if a == b and a < 4:
                match += 1
            elif a < 4 and b < 4 and (a ^ b) == 2:
                ts += 1
            else:
                tv += 1
        near = wide = 0
        down = up = None
        for y in range(n):
            if y == x:
                continue
            dt = ta[y] - ta[x]
            if abs(dt) <= WIDE_T:
                wide += 1
            if abs(dg[y] - dg[x]) <= NEAR_DIAG:
                if abs(dt) <= NEAR_T:
                    near += 1
                if 0 < dt <= WIDE_T and (down is None or dt < down):
                    down = dt
                if -WIDE_T <= dt < 0 and (up is None or -dt < up):
                    up = -dt
        out[x] = [
            sc / 4096.0,
            np.log2(1 + L) / 16.0,
            match / L,
            ts / L,
            tv / L,
            (t0 - q0) / nt,
            float(strand),
            ta[x] / nt,
            qa[x] / nq,
            _gc(tc, ta[x] - GC_W, ta[x] + GC_W),
            _gc(qc, qa[x] - GC_W, qa[x] + GC_W),
            np.log2(1 + near) / 8.0,
            np.log2(1 + wide) / 8.0,
            np.log2(1 + down) / 16.0 if down is not None else 1.0,
            np.log2(1 + up) / 16.0 if up is not None else 1.0,
            _soft(tsoft, ta[x] - GC_W, ta[x] + GC_W),
        ]
    return out


def targets(fwd, bwd):
    """Regression targets of one extension from its two halves, each a tuple
    (cells, i_end, j_end): log2(1 + cells) and log2(1 + i* + j*), forward half
    first."""
    return np.array([np.log2(1 + fwd[0]), np.log2(1 + fwd[1] + fwd[2]),
                     np.log2(1 + bwd[0]), np.log2(1 + bwd[1] + bwd[2])], dtype=np.float64)
