"""The allocation-free gradient entry point (sfe_model_grad_noalloc) through
the C ABI: its output equals sfe_model_grad's, bit for bit, on two calls in a
row (the second smaller, so stale working memory would show), and it refuses
sizes beyond its fixed working memory and host buffers."""
import numpy as np
import pytest

from paper_2606_06811_amd import sfe

pytestmark = pytest.mark.gpu


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)


def init_params(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in ((64, 16), (64, 64), (64, 64), (4, 64)):
        lim = np.sqrt(6.0 / i)
        parts += [rng.uniform(-lim, lim, o * i), np.zeros(o)]
    return np.concatenate(parts).astype(np.float32)


def test_grad_noalloc_equals_grad():
    import torch
    log("no-alloc gradient: context and model on device 0")
    dev = torch.device("cuda:0")
    ctx = sfe.sfe_ctx_create(0)
    m = sfe.Model(ctx, init_params(21))
    rng = np.random.default_rng(22)
    try:
        for n in (5000, 777):
            log(f"no-alloc gradient with {n} samples")
            X = rng.uniform(0, 1, (n, sfe.MLP_NFEAT)).astype(np.float32)
            T = rng.uniform(0, 14, (n, sfe.MLP_NOUT)).astype(np.float32)
            ref_loss, ref_g = m.grad(X, T)
            xd = torch.from_numpy(X).to(dev)
            td = torch.from_numpy(T).to(dev)
            gd = torch.full((sfe.MLP_NPARAMS,), float("nan"), dtype=torch.float32, device=dev)
            ld = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
            torch.cuda.synchronize()
            m.grad_noalloc(xd, td, gd, ld)
            torch.cuda.synchronize()
            g = gd.cpu().numpy()
            assert np.array_equal(g, ref_g), float(np.abs(g - ref_g).max())
            assert float(ld.cpu().numpy()[0]) == ref_loss
        # beyond the fixed working memory, and host buffers, are refused
        big = torch.zeros((sfe.NOALLOC_MAX_SAMPLES + 1, sfe.MLP_NFEAT), dtype=torch.float32, device=dev)
        bt = torch.zeros((sfe.NOALLOC_MAX_SAMPLES + 1, sfe.MLP_NOUT), dtype=torch.float32, device=dev)
        with pytest.raises(sfe.SfeError) as e:
            m.grad_noalloc(big, bt, gd, ld)
        assert e.value.status == sfe.SFE_EINVAL
        with pytest.raises(sfe.SfeError) as e:
            m.grad_noalloc(X, T, gd, ld)
        assert e.value.status == sfe.SFE_EINVAL
    finally:
        m.close()
        ctx.close()
