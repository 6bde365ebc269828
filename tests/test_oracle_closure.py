"""Pins of the closure network's oracle: finite-difference gradients, the
bfloat16 rounding it emulates, and the feature definition on fields whose
stencil differences are known."""

import numpy as np
import pytest
import torch

from oracle import closure as C


@pytest.mark.parametrize("act", [C.TANH, C.RELU])
def test_gradient_matches_finite_differences(act):
    rng = np.random.default_rng(0)
    p = C.init_params(seed=3).astype(np.float64)
    p[C.OB1:C.OW2] = rng.normal(0, 0.1, C.HID)
    p[C.OB3:C.OB3 + 4] = rng.normal(0, 0.1, 4)
    X = rng.normal(0, 1, (40, C.KIN))
    T = rng.normal(0, 1, (40, 4))
    loss, g = C.loss_and_grad(p, X, T, act=act)
    picks = np.concatenate([rng.choice(np.arange(C.OW1, C.OB1), 12), rng.choice(np.arange(C.OB1, C.OW2), 4),
                            rng.choice(np.arange(C.OW2, C.OB2), 12), rng.choice(np.arange(C.OB2, C.OW3), 4),
                            rng.choice(np.arange(C.OW3, C.OW3 + 4 * C.HID), 8), np.arange(C.OB3, C.OB3 + 4)])
    for q in picks:
        h = 1e-6 * max(1.0, abs(p[q]))
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd = (C.loss_and_grad(pp, X, T, act=act)[0] - C.loss_and_grad(pm, X, T, act=act)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1e-3, abs(g[q])) + 1e-10, (q, fd, g[q])
    if act == C.RELU:   # both layers have units on each side of the kink
        _, H1, H2, _ = C.forward(p, X, act=act)
        assert 0.2 < (H1 > 0).mean() < 0.8 and 0.2 < (H2 > 0).mean() < 0.8
    # unused padded outputs get no gradient
    assert np.all(g[C.OW3 + 4 * C.HID:C.OB3] == 0.0) and np.all(g[C.OB3 + 4:] == 0.0)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 3, 5000), [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 65504.0, 1e-30]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16(x), ref)


def test_features_of_linear_and_constant_fields():
    """On a linear field f = a x + b z the slot-k features are
    (a dx_k + b dz_k) / scale; on a constant field they vanish (slot 0 holds
    the value itself)."""
    nx = 7
    xy = np.array([[i, j] for j in range(nx) for i in range(nx)], float)
    idx = np.array([[c] + [j for j in np.argsort(((xy - xy[c]) ** 2).sum(1), kind="stable") if j != c][:36]
                    for c in range(nx * nx)])
    E = 2
    st = np.zeros((nx * nx, E, 4))
    st[:, 0, 0] = 2.0 * xy[:, 0] - 3.0 * xy[:, 1]
    st[:, 1, 2] = 7.0
    nodef = xy[:, 1] / 6.0
    scale = [2.0, 1.0, 7.0, 1.0]
    X = C.features(st, idx, nodef, scale).reshape(nx * nx, E, C.KIN)
    for c in (0, 17, 48):
        d = xy[idx[c]] - xy[c]
        np.testing.assert_allclose(X[c, 0, 4:4 * 37:4], (2.0 * d[1:, 0] - 3.0 * d[1:, 1]) / 2.0)
        assert X[c, 1, 2] == 1.0 and np.all(X[c, 1, 6:4 * 37:4] == 0.0)
        assert X[c, 0, 148] == nodef[c] and np.all(X[c, :, 149:] == 0.0)
