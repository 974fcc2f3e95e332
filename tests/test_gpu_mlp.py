"""Cost-model kernels (FP32, GPU) against the FP64 oracle.

FP32 sums in a different order than the FP64 reference, so the comparison is
to a tolerance: forward |dy| <= 1e-4 (1 + |y|); gradients within 1e-3 of the
reference gradient's norm; Adam steps and short training runs stay within
the same relative bound."""
import numpy as np
import pytest
import torch

import moma_inputs as mi

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def data(rows, seed):
    x = mi.uniform01(rows * mi.MLP_IN, 91, seed).reshape(rows, mi.MLP_IN) * 4 - 2
    t = np.sin(x[:, 0]) + 0.3 * x[:, 1] * x[:, 2] + 0.1 * x.sum(axis=1)
    return x, t


def test_nparams_agree():
    import oracle
    import paper_2501_07535_amd as moma
    assert moma.mlp_nparams() == oracle.mlp_nparams() == mi.MLP_NPARAM


@pytest.mark.parametrize("rows", [1, 7, 300, 4097])
def test_forward_matches_oracle(rows):
    import oracle
    import paper_2501_07535_amd as moma
    p = mi.mlp_init(11)
    p[64 * mi.MLP_IN:64 * (mi.MLP_IN + 1)] = 0.02
    p32 = p.astype(np.float32).astype(np.float64)
    x, _ = data(rows, rows)
    x32 = x.astype(np.float32).astype(np.float64)
    y = torch.zeros(rows, dtype=torch.float32, device="cuda:0")
    moma.mlp_forward(dev(p), dev(x), y)
    want = oracle.mlp_forward(p32, x32)
    got = y.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= 1e-4 * (1 + np.abs(want)))


@pytest.mark.parametrize("rows", [3, 256, 2000])
def test_gradient_matches_oracle(rows):
    import oracle
    import paper_2501_07535_amd as moma
    p = mi.mlp_init(12)
    p[64 * mi.MLP_IN:64 * (mi.MLP_IN + 1)] = 0.02
    p32 = p.astype(np.float32).astype(np.float64)
    x, t = data(rows, 100 + rows)
    x32, t32 = x.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
    g = torch.zeros(mi.MLP_NPARAM, dtype=torch.float32, device="cuda:0")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    moma.mlp_grad(dev(p), dev(x), dev(t), g, loss)
    gw, lw = oracle.mlp_grad(p32, x32, t32)
    gg = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - lw) <= 1e-4 * (1 + lw)
    assert np.linalg.norm(gg - gw) <= 1e-3 * np.linalg.norm(gw)
    big = np.abs(gw) > 1e-3 * np.abs(gw).max()
    assert np.all(np.abs(gg[big] - gw[big]) <= 1e-3 * np.abs(gw[big]) + 1e-5 * np.abs(gw).max())


def test_adam_and_training_track_oracle():
    import oracle
    import paper_2501_07535_amd as moma
    p = mi.mlp_init(13).astype(np.float32).astype(np.float64)
    x, t = data(512, 13)
    x, t = x.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
    dp, dx, dt = dev(p), dev(x), dev(t)
    g = torch.zeros_like(dp)
    m, v = torch.zeros_like(dp), torch.zeros_like(dp)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    pr, mr, vr = p.copy(), np.zeros_like(p), np.zeros_like(p)
    first = None
    for step in range(1, 41):
        moma.mlp_grad(dp, dx, dt, g, loss)
        moma.mlp_adam(dp, g, m, v, step, 2e-3)
        gr, lr_ = oracle.mlp_grad(pr, x, t)
        oracle.mlp_adam(pr, gr, mr, vr, step, 2e-3)
        first = first if first is not None else lr_
    torch.cuda.synchronize()
    pg = dp.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(pg - pr) <= 1e-3 * np.linalg.norm(pr)
    assert oracle.mlp_grad(pr, x, t)[1] < first
