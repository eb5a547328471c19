"""Pins of the oracle's MLP (the learned h-seed; not part of the paper).

The FP64 gradient is checked against central finite differences of the loss;
bfloat16 rounding against hand-picked values; Adam against a hand-computed
first step."""
import numpy as np
import pytest

import oracle


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, oracle.MLP_NPARAM)


def test_layout_size():
    assert sum(int(np.prod(s)) for _, s in oracle.MLP_SIZES) == oracle.MLP_NPARAM == 4801
    p = _params(0)
    np.testing.assert_array_equal(oracle.mlp_pack(oracle.mlp_unpack(p)), p)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = _params(2)
    feat = rng.normal(0, 1, (37, 8))
    t = rng.normal(0, 0.5, 37)
    loss, g = oracle.mlp_loss_grad(p, feat, t)
    eps = 1e-6
    idx = np.concatenate([rng.choice(np.arange(0, 512), 40, replace=False),      # W1
                          rng.choice(np.arange(512, 576), 10, replace=False),    # b1
                          rng.choice(np.arange(576, 4672), 60, replace=False),   # W2
                          rng.choice(np.arange(4672, 4736), 10, replace=False),  # b2
                          rng.choice(np.arange(4736, 4800), 10, replace=False),  # w3
                          [4800]])                                               # b3
    fd = []
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += eps
        pm[k] -= eps
        fd.append((oracle.mlp_loss_grad(pp, feat, t)[0] - oracle.mlp_loss_grad(pm, feat, t)[0]) / (2 * eps))
    fd = np.array(fd)
    err = np.abs(fd - g[idx])
    assert np.all(err <= 1e-6 * np.maximum(1.0, np.abs(fd)) + 1e-7), (err.max(), idx[err.argmax()])


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 0.0, 1.0 + 2 ** -7 + 2 ** -12])
    got = oracle.bf16(vals)
    # bfloat16 keeps 8 significant bits: 1 + 2^-8 is a tie between 1 and
    # 1 + 2^-7 (even: 1); 1 + 3*2^-8 ties between 1 + 2^-7 and 1 + 2^-6 (even:
    # 1 + 2^-6); 1 + 2^-7 + 2^-12 is nearest to 1 + 2^-7
    np.testing.assert_array_equal(got, [1.0, 1.0, 1.0 + 2 ** -6, 1.0, -2.5, 0.0, 1.0 + 2 ** -7])
    bits = got.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)


def test_quantised_forward_close_to_exact():
    rng = np.random.default_rng(3)
    p = _params(4)
    feat = rng.normal(0, 1, (200, 8))
    y0, _ = oracle.mlp_forward(p, feat, False)
    y1, _ = oracle.mlp_forward(p, feat, True)
    assert np.abs(y1 - y0).max() < 0.05 * (np.abs(y0).max() + 1)


def test_adam_first_step():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -4.0])
    p1, m, v = oracle.adam_step(p, g, np.zeros(2), np.zeros(2), 1, 0.01)
    # first bias-corrected step moves every parameter by lr * sign(g) (up to eps)
    np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-9)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    rng = np.random.default_rng(5)
    feat = rng.normal(0, 1, (512, 8))
    t = np.tanh(feat[:, 0]) - 0.3 * feat[:, 1] ** 2 + 0.1
    p = _params(6, 0.1)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = oracle.mlp_loss_grad(p, feat, t)[0]
    for step in range(1, 301):
        loss, g = oracle.mlp_loss_grad(p, feat, t)
        p, m, v = oracle.adam_step(p, g, m, v, step, 3e-3)
    assert oracle.mlp_loss_grad(p, feat, t)[0] < 0.2 * l0
