"""CPU oracle of the learned coarse closure's network. TEST INFRASTRUCTURE ONLY.

The network is not in the paper: it is a learned correction to the coarse
right-hand side, defined by the closure interface of the C ABI. For node i
and member e the input is the stencil-gathered state -- slot 0 the node's own
fields, slots k >= 1 the differences f(j_k) - f(i), each field divided by its
input scale -- plus one per-node value, zero-padded to 160; then
h1 = a(W1 x + b1), h2 = a(W2 h1 + b2), y = W3 h2 + b3 (128 hidden, 4 outputs)
with the activation a = tanh or a = relu (max(v, 0)); loss = mean over
samples and outputs of (y - target)^2.

Everything here is FP64. With ``emulate=True`` the values the GPU stores in
bfloat16 (inputs, weights, hidden activations and back-propagated
activations) are rounded to bfloat16 at the same places, and the output-layer
gradient to FP32, so the GPU can be compared at FP32-accumulation accuracy;
with ``emulate=False`` it is the plain FP64 network, whose analytic gradient
is pinned by finite differences. The two differ only by those roundings
(pinned: with the roundings replaced by the identity they agree bit for bit,
and a hand-computed two-sample case fixes where each rounding happens).
"""

import numpy as np

HID, KIN, NOUT, NSLOT = 128, 160, 16, 37
TANH, RELU = 0, 1


def _act(v, act):
    return np.tanh(v) if act == TANH else np.maximum(v, 0.0)


def _dact(h, act):
    """Derivative of the activation expressed through its output h."""
    return 1.0 - h * h if act == TANH else (h > 0.0).astype(np.float64)
OW1 = 0
OB1 = OW1 + HID * KIN
OW2 = OB1 + HID
OB2 = OW2 + HID * HID
OW3 = OB2 + HID
OB3 = OW3 + NOUT * HID
NPARAM = OB3 + NOUT


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as FP64. The
    value is first rounded to FP32, as the GPU computes in FP32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def fp32(x):
    """Round to the nearest FP32, returned as FP64."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _exact(x):
    return np.asarray(x, dtype=np.float64)


def _rounders(emulate):
    """(r16, r32): the roundings applied where the GPU stores a value --
    bfloat16 for the matrix-core operands and activations, FP32 for the
    output-layer gradient -- or no rounding for the plain network."""
    return (bf16, fp32) if emulate else (_exact, _exact)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[OW1:OB1].reshape(HID, KIN), p[OB1:OW2], p[OW2:OB2].reshape(HID, HID), p[OB2:OW3],
            p[OW3:OB3].reshape(NOUT, HID), p[OB3:NPARAM])


def features(state, idx, node_feature, in_scale):
    """X [n_active * E][160] from state [n_total][E][4] and stencils
    idx [n_active][n] (slot 0 = the node itself)."""
    na, n = idx.shape
    E = state.shape[1]
    sc = 1.0 / np.asarray(in_scale, dtype=np.float64)
    X = np.zeros((na, E, KIN))
    own = state[:na]                                         # [na][E][4]
    X[:, :, 0:4] = own * sc
    for k in range(1, n):
        X[:, :, 4 * k:4 * k + 4] = (state[idx[:, k]] - own) * sc
    X[:, :, 4 * NSLOT] = np.asarray(node_feature)[:, None]
    return X.reshape(na * E, KIN)


def forward(p, X, emulate=False, act=TANH):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    r, _ = _rounders(emulate)
    Xr, W1r, W2r, W3r = r(X), r(W1), r(W2), r(W3)
    H1 = r(_act(Xr @ W1r.T + b1, act))
    H2 = r(_act(H1 @ W2r.T + b2, act))
    Y = H2 @ W3r.T + b3
    return Y, H1, H2, Xr


def loss_and_grad(p, X, T, emulate=False, act=TANH):
    """Loss and its gradient for targets T [S][4] (only outputs 0..3 enter)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    r, r32 = _rounders(emulate)
    Y, H1, H2, Xr = forward(p, X, emulate, act)
    S = X.shape[0]
    D = Y[:, :4] - T
    loss = float(np.sum(D * D) / (4 * S))
    dY32 = np.zeros((S, NOUT))
    dY32[:, :4] = 2.0 * D / (4 * S)
    dY32 = r32(dY32)
    dY = r(dY32)
    dH2 = r((dY @ r(W3)) * _dact(H2, act))
    dH1 = r((dH2 @ r(W2)) * _dact(H1, act))
    g = np.zeros(NPARAM)
    g[OW1:OB1] = (dH1.T @ Xr).ravel()
    g[OB1:OW2] = dH1.sum(axis=0)
    g[OW2:OB2] = (dH2.T @ H1).ravel()
    g[OB2:OW3] = dH2.sum(axis=0)
    g[OW3:OB3] = (dY.T @ H2).ravel()
    g[OB3:NPARAM] = dY32.sum(axis=0)
    return loss, g


def init_params(seed=0, out_rows=4):
    """Seeded initial parameters: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in))
    weights, zero biases; W3 rows beyond the 4 outputs are zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(NPARAM)
    p[OW1:OB1] = rng.uniform(-1, 1, HID * KIN) / np.sqrt(149.0)
    p[OW2:OB2] = rng.uniform(-1, 1, HID * HID) / np.sqrt(HID)
    w3 = np.zeros((NOUT, HID))
    w3[:out_rows] = rng.uniform(-1, 1, (out_rows, HID)) / np.sqrt(HID)
    p[OW3:OB3] = w3.ravel()
    return p.astype(np.float32)
