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


@pytest.mark.parametrize("act", [C.TANH, C.RELU])
def test_emulation_is_the_plain_network_plus_roundings(act, monkeypatch):
    """With every emulated rounding replaced by the identity, the emulated
    network and its gradient equal the plain FP64 network's bit for bit: the
    emulation changes nothing but the stored precisions."""
    rng = np.random.default_rng(8)
    p = C.init_params(seed=6).astype(np.float64)
    p[C.OB1:C.OW2] = rng.normal(0, 0.1, C.HID)
    X = rng.normal(0, 1, (30, C.KIN))
    T = rng.normal(0, 1, (30, 4))
    y_plain = C.forward(p, X, emulate=False, act=act)[0]
    l_plain, g_plain = C.loss_and_grad(p, X, T, emulate=False, act=act)
    assert not np.array_equal(C.forward(p, X, emulate=True, act=act)[0], y_plain)
    ident = lambda v: np.asarray(v, dtype=np.float64)  # noqa: E731
    monkeypatch.setattr(C, "bf16", ident)
    monkeypatch.setattr(C, "fp32", ident)
    assert np.array_equal(C.forward(p, X, emulate=True, act=act)[0], y_plain)
    l_em, g_em = C.loss_and_grad(p, X, T, emulate=True, act=act)
    assert l_em == l_plain and np.array_equal(g_em, g_plain)


def test_emulated_roundings_by_hand():
    """Two samples through one active hidden unit per layer (relu), with
    values chosen so that each stored quantity -- input, W1, first hidden
    activation, W2, second hidden activation, W3, output gradient and both
    back-propagated activations -- rounds visibly to bfloat16 (8 significant
    bits, ties to even), while pre-activations, biases and outputs do not.
    Every expected value below was worked out by hand."""
    p = np.zeros(C.NPARAM)
    p[C.OW1] = 1 + 2 ** -9            # W1[0,0] -> 1.0
    p[C.OB1] = 2 ** -10               # b1[0], kept exact
    p[C.OW2] = 3 + 2 ** -7            # W2[0,0]: a tie -> 3.0 (even)
    p[C.OB2] = 2 ** -10
    p[C.OW3] = 1.5 + 2 ** -9          # W3[0,0] -> 1.5
    p[C.OB3] = 0.25
    X = np.zeros((2, C.KIN))
    X[:, 0] = [1 + 2 ** -8, 1 + 3 * 2 ** -9]   # -> 1.0 (a tie, to even) and 1.0078125
    Y, H1, H2, Xr = C.forward(p, X, emulate=True, act=C.RELU)
    assert Xr[:, 0].tolist() == [1.0, 1.0078125]
    # pre-activation 1 + 2^-10 and 1.0078125 + 2^-10 stored as bfloat16
    assert H1[:, 0].tolist() == [1.0, 1.0078125] and np.all(H1[:, 1:] == 0.0)
    # 3 x H1 + 2^-10: 3.0009765625 -> 3.0 and 3.0244140625 -> 3.03125
    assert H2[:, 0].tolist() == [3.0, 3.03125] and np.all(H2[:, 1:] == 0.0)
    # 1.5 x H2 + 0.25, not rounded
    assert Y[:, 0].tolist() == [4.75, 4.796875] and np.all(Y[:, 1:4] == 0.0)
    # targets giving output gradients (Y - T) / 4 = 1 + 2^-8 + 2^-10 and 1/8
    T = np.zeros((2, 4))
    T[:, 0] = [4.75 - 4 * (1 + 2 ** -8 + 2 ** -10), 4.796875 - 0.5]
    loss, g = C.loss_and_grad(p, X, T, emulate=True, act=C.RELU)
    assert loss == 2.0508289337158203125              # 2 (1.0048828125^2 + 0.125^2)
    # dY: 1.0048828125 -> 1.0078125; dH2 = 1.5 dY: 1.51171875 (a tie) -> 1.515625,
    # 0.1875; dH1 = 3 dH2: 4.546875 (a tie) -> 4.5625, 0.5625
    assert g[C.OW1] == 4.5625 * 1.0 + 0.5625 * 1.0078125       # 5.12939453125
    assert g[C.OB1] == 5.125
    assert g[C.OW2] == 1.515625 * 1.0 + 0.1875 * 1.0078125     # 1.70458984375
    assert g[C.OB2] == 1.703125
    assert g[C.OW3] == 1.0078125 * 3.0 + 0.125 * 3.03125       # 3.40234375
    assert g[C.OB3] == 1.0048828125 + 0.125                    # output-bias gradient: FP32, not bfloat16
    nz = np.flatnonzero(g)
    assert sorted(nz.tolist()) == sorted([C.OW1, C.OB1, C.OW2, C.OB2, C.OW3, C.OB3])
    # the plain network on the same case rounds nowhere
    Yp = C.forward(p, X, emulate=False, act=C.RELU)[0]
    assert Yp[0, 0] == 1.5019531250 * (3.0078125 * ((1 + 2 ** -8) * (1 + 2 ** -9) + 2 ** -10) + 2 ** -10) + 0.25
