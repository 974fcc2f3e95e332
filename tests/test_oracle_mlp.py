"""Pins for the FP64 MLP oracle (CPU only): finite differences, the all-active
linear case against numpy matrix products, the zero-weight case, the closed
form of the first Adam step, and that training lowers the loss."""
import numpy as np
import pytest

import moma_inputs as mi

NP = mi.MLP_NPARAM


def split(p):
    o = 0
    out = []
    for n in (64 * mi.MLP_IN, 64, 64 * 64, 64, 64, 1):
        out.append(p[o:o + n])
        o += n
    W1, b1, W2, b2, W3, b3 = out
    return W1.reshape(64, mi.MLP_IN), b1, W2.reshape(64, 64), b2, W3, b3


def data(rows, seed):
    x = mi.uniform01(rows * mi.MLP_IN, 77, seed).reshape(rows, mi.MLP_IN) * 4 - 2
    t = mi.uniform01(rows, 78, seed) * 3
    return x, t


def test_nparams():
    import oracle
    assert oracle.mlp_nparams() == NP == 64 * 7 + 64 + 64 * 64 + 64 + 64 + 1 == 4737


def test_gradient_matches_central_differences():
    import oracle
    p = mi.mlp_init(1)
    p[64 * mi.MLP_IN:64 * (mi.MLP_IN + 1)] = 0.05            # small positive biases: fewer units sit exactly at the ReLU kink
    x, t = data(32, 1)
    g, loss = oracle.mlp_grad(p, x, t)
    idx = np.unique(np.concatenate([np.arange(NP - 70, NP), np.random.default_rng(0).integers(0, NP, 400)]))
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        num = (oracle.mlp_grad(pp, x, t)[1] - oracle.mlp_grad(pm, x, t)[1]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)) + 1e-9, (i, num, g[i])


def test_all_active_network_is_a_matrix_product():
    import oracle
    rng = np.random.default_rng(2)
    p = np.concatenate([rng.uniform(0.01, 0.2, 64 * mi.MLP_IN), rng.uniform(0.1, 0.3, 64), rng.uniform(0.01, 0.05, 64 * 64),
                        rng.uniform(0.1, 0.3, 64), rng.uniform(-1, 1, 64), [0.7]])
    x = rng.uniform(0.1, 2.0, (50, mi.MLP_IN))
    W1, b1, W2, b2, W3, b3 = split(p)
    want = ((x @ W1.T + b1) @ W2.T + b2) @ W3 + b3
    assert np.allclose(oracle.mlp_forward(p, x), want, rtol=1e-13, atol=1e-13)


def test_zero_weights():
    import oracle
    p = np.zeros(NP)
    p[-1] = 1.5
    x, t = data(40, 3)
    assert np.all(oracle.mlp_forward(p, x) == 1.5)
    g, loss = oracle.mlp_grad(p, x, t)
    assert loss == pytest.approx(np.mean((1.5 - t) ** 2), rel=1e-14)
    assert g[-1] == pytest.approx(2 * np.mean(1.5 - t), rel=1e-12)
    assert np.all(g[:-1] == 0)


def test_first_adam_step_closed_form():
    import oracle
    p = mi.mlp_init(4)
    g = np.random.default_rng(4).normal(size=NP)
    m, v = np.zeros(NP), np.zeros(NP)
    q = p.copy()
    oracle.mlp_adam(q, g, m, v, 1, 1e-2)
    # bias-corrected first moments equal g and g^2, so the step is lr * g / (|g| + eps)
    assert np.allclose(q, p - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_lowers_the_loss():
    import oracle
    p = mi.mlp_init(5)
    x, _ = data(256, 5)
    t = x.sum(axis=1) * 0.5 + np.sin(x[:, 0])
    m, v = np.zeros(NP), np.zeros(NP)
    first = oracle.mlp_grad(p, x, t)[1]
    for step in range(1, 301):
        g, loss = oracle.mlp_grad(p, x, t)
        oracle.mlp_adam(p, g, m, v, step, 3e-3)
    assert loss < first / 20


def test_init_statistics():
    p = mi.mlp_init(6)
    W1, b1, W2, b2, W3, b3 = split(p)
    assert np.all(b1 == 0) and np.all(b2 == 0) and b3[0] == 0
    assert abs(W2.std() - np.sqrt(2 / 64)) < 0.02
    assert abs(W2.mean()) < 0.02
    assert np.array_equal(p, mi.mlp_init(6))
