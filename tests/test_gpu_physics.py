"""The paper's density current (Section 6.4) through the whole GPU path --
stencil search, weights, ghost closure, fused RHS, RK4 to t = 900 s -- at
100 m on the three node layouts, against Table tbl:straka's 100 m rows.

The run differs from the paper's only where the paper is silent or garbled
(hyperviscosity amount, ghost placement; see the design notes), so the
comparison is at percent level, not parity."""

import csv
import os

import numpy as np
import pytest

import oracle as O
from workloads import density_current_config, bubble_config

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def table_row(layout, h):
    with open(os.path.join(GOLDEN, "straka_table.csv")) as f:
        rows = [r for r in csv.reader(f) if r and not r[0].startswith("#")][1:]
    return {(r[0], float(r[1])): [float(v) for v in r[2:]] for r in rows}[layout, h]


@pytest.mark.parametrize("layout,fdt", [("hexagonal", 0), ("cartesian", 0), ("scattered", 0), ("hexagonal", 1)])
def test_density_current_100m_against_table(layout, fdt):
    import torch
    from paper_1509_02615_amd import rbffd as R
    from paper_1509_02615_amd import pipeline as P
    print(f"density current: {layout} 100 m, field dtype {fdt}, RK4 3600 steps", flush=True)
    ctx = R.Context(0)
    cfg = density_current_config(layout, 100.0)
    nd = cfg["nodes"]
    xy, idx, W, Ww, (sa, sw) = P.ns_weights(ctx, cfg)
    assert int(sa.abs().sum()) == 0 and int(sw.abs().sum()) == 0
    model = P.ns_model(ctx, cfg, idx, W, Ww, xy=xy, field_dtype=fdt, weight_dtype=fdt)
    dt = torch.float64 if fdt == 0 else torch.float32
    s = P.to_dev(cfg["state0"], dt).reshape(model.state_shape()).contiguous()
    t = 0.0
    for _ in range(6):
        t = R.rbffd_step(ctx, model, s, t, cfg["dt"], 600, R.RK4)
        print(f"   t = {t:.0f} s", flush=True)
    assert abs(t - 900.0) < 1e-9
    R.rbffd_ghost(ctx, model, s)
    y = s.double().cpu().numpy().reshape(-1, 4)
    e = O.extrema(y, nd.n_active)
    front = O.front_location(nd.xy, y[:, 2], nd.wall_nodes[0])
    got = [e["theta_min"], e["theta_max"], e["w_min"], e["w_max"], front]
    ref = table_row(layout, 100.0)
    print(f"   layout {layout}: got {np.round(got, 2).tolist()} table {ref}", flush=True)
    # extrema of theta' and w' within 5% (+0.15 K / m s^-1 absolute for the small max theta'),
    # front within 1.5%
    for g, r in zip(got[:4], ref[:4]):
        assert abs(g - r) <= 0.05 * abs(r) + 0.15, (got, ref)
    assert abs(front - ref[4]) <= 0.015 * ref[4], (front, ref[4])


def translating_row(layout, h):
    with open(os.path.join(GOLDEN, "translating_table.csv")) as f:
        rows = [r for r in csv.reader(f) if r and not r[0].startswith("#")][1:]
    return {(r[0], float(r[1])): [float(v) for v in r[2:]] for r in rows}[layout, h]


@pytest.mark.parametrize("layout", ["hexagonal", "cartesian"])
def test_translating_density_current_100m_against_table(layout):
    import torch
    from paper_1509_02615_amd import rbffd as R
    from paper_1509_02615_amd import pipeline as P
    from workloads import translating_config
    print(f"translating density current: {layout} 100 m, u_bar = 20 m/s, RK4 3600 steps", flush=True)
    ctx = R.Context(0)
    cfg = translating_config(layout, 100.0)
    nd = cfg["nodes"]
    xy, idx, W, Ww, (sa, sw) = P.ns_weights(ctx, cfg)
    model = P.ns_model(ctx, cfg, idx, W, Ww, xy=xy)
    s = P.to_dev(cfg["state0"], torch.float64).reshape(model.state_shape()).contiguous()
    t = 0.0
    for _ in range(6):
        t = R.rbffd_step(ctx, model, s, t, cfg["dt"], 600, R.RK4)
    R.rbffd_ghost(ctx, model, s)
    y = s.cpu().numpy().reshape(-1, 4)
    left, right = O.translating_fronts(nd.xy, y[:, 2], nd.wall_nodes[0])
    ref = translating_row(layout, 100.0)
    print(f"   layout {layout}: fronts (left, right) from 18 km {left:.0f} {right:.0f} table {ref}", flush=True)
    assert abs(left - ref[0]) <= 0.03 * ref[0] and abs(right - ref[1]) <= 0.03 * ref[1]


def bubble_row(layout, h):
    with open(os.path.join(GOLDEN, "bubble_table.csv")) as f:
        rows = [r for r in csv.reader(f) if r and not r[0].startswith("#")][1:]
    return {(r[0], float(r[1])): [float(v) for v in r[2:]] for r in rows}[layout, h]


def run_bubble(layout, h, fdt=0):
    import torch
    from paper_1509_02615_amd import rbffd as R
    from paper_1509_02615_amd import pipeline as P
    ctx = R.Context(0)
    cfg = bubble_config(layout, h)
    nd = cfg["nodes"]
    xy, idx, W, Ww, (sa, sw) = P.ns_weights(ctx, cfg)
    assert int(sa.abs().sum()) == 0 and int(sw.abs().sum()) == 0
    model = P.ns_model(ctx, cfg, idx, W, Ww, xy=xy, field_dtype=fdt, weight_dtype=fdt)
    s = P.to_dev(cfg["state0"], torch.float64 if fdt == 0 else torch.float32).reshape(model.state_shape()).contiguous()
    n = int(round(cfg["t_end"] / cfg["dt"]))
    t = R.rbffd_step(ctx, model, s, 0.0, cfg["dt"], n, R.RK4)
    assert abs(t - 1100.0) < 1e-9
    R.rbffd_ghost(ctx, model, s)
    y = s.double().cpu().numpy().reshape(-1, 4)
    na = nd.n_active
    got = [y[:na, 2].min(), y[:na, 2].max(), y[:na, 1].min(), y[:na, 1].max(),
           O.bubble_height(nd.xy, y[:, 2], nd.rows)]
    return cfg, y, got


@pytest.mark.parametrize("layout,h,fdt", [("cartesian", 200.0, 0), ("hexagonal", 200.0, 0), ("scattered", 200.0, 0),
                                          ("cartesian", 100.0, 0), ("hexagonal", 100.0, 0),
                                          ("scattered", 100.0, 0), ("cartesian", 100.0, 1)])
def test_rising_bubble_against_table(layout, h, fdt):
    """Section 6.5 (mu = 10 m^2/s, t = 1100 s) through the whole GPU path,
    four-wall ghost closure included, against Table tbl:bubble: max theta'
    and the w' extrema within 12%, min theta' (~ -0.1 K) within 0.05 K, the
    bubble height within 2.5%."""
    print(f"rising bubble: {layout} {h} m, field dtype {fdt}", flush=True)
    cfg, y, got = run_bubble(layout, h, fdt)
    ref = bubble_row(layout, h)
    print(f"   got {np.round(got, 3).tolist()} table {ref}", flush=True)
    assert abs(got[0] - ref[0]) <= 0.05
    for k in (1, 2, 3):
        assert abs(got[k] - ref[k]) <= 0.12 * abs(ref[k]), (k, got, ref)
    assert abs(got[4] - ref[4]) <= 0.025 * ref[4], (got, ref)


def _shared_errors(ref_cfg, ref_y, runs, spacing):
    """theta' relative l2 of each (cfg, y) run against the reference run, on
    the nodes of the `spacing` lattice (which every grid holds)."""
    rxy = ref_cfg["nodes"].xy[:ref_cfg["nodes"].n_active]
    key = {(round(x, 3), round(z, 3)): i for i, (x, z) in enumerate(rxy)}
    errs = []
    for cfg, y in runs:
        nd = cfg["nodes"]
        x0 = nd.xy[:nd.n_active, 0].min()
        common = [(i, key[(round(x, 3), round(z, 3))]) for i, (x, z) in enumerate(nd.xy[:nd.n_active])
                  if (round(x, 3), round(z, 3)) in key and abs((x - x0) % spacing) < 1e-6 and abs(z % spacing) < 1e-6]
        a = np.array([y[i, 2] for i, _ in common])
        b = np.array([ref_y[j, 2] for _, j in common])
        errs.append(np.linalg.norm(a - b) / np.linalg.norm(b))
    return errs


def test_rising_bubble_converges():
    """Section 6.5: Cartesian nodes at 400, 200, 100, 50 and 25 m against a
    12.5 m run of the same method (dt halving with h: 1/32 s), theta'
    compared on the 400 m nodes (which every grid holds). The error falls
    with every halving of h, and below 100 m at high order: above 2.2 from
    100 to 50 m and above 3 from 50 to 25 m (the paper: second order down to
    100 m, fourth below)."""
    ref_cfg, ref_y, _ = run_bubble("cartesian", 12.5)
    hs = (400.0, 200.0, 100.0, 50.0, 25.0)
    runs = [run_bubble("cartesian", h)[:2] for h in hs]
    errs = _shared_errors(ref_cfg, ref_y, runs, 400.0)
    orders = [np.log2(errs[k] / errs[k + 1]) for k in range(len(hs) - 1)]
    print(f"   theta' rel-l2 vs 12.5 m at {hs} m: {['%.2e' % e for e in errs]}, "
          f"orders {['%.2f' % o for o in orders]}", flush=True)
    # measured: errors 0.517, 0.334, 0.148, 0.0257, 0.00264; orders 0.63, 1.18, 2.52, 3.28
    assert all(errs[k + 1] < errs[k] for k in range(len(hs) - 1))
    assert orders[-1] > 3.0 and orders[-2] > 2.2


def run_density_current(layout, h):
    import torch
    from paper_1509_02615_amd import rbffd as R
    from paper_1509_02615_amd import pipeline as P
    ctx = R.Context(0)
    cfg = density_current_config(layout, h)
    xy, idx, W, Ww, (sa, sw) = P.ns_weights(ctx, cfg)
    assert int(sa.abs().sum()) == 0 and int(sw.abs().sum()) == 0
    model = P.ns_model(ctx, cfg, idx, W, Ww, xy=xy)
    s = P.to_dev(cfg["state0"], torch.float64).reshape(model.state_shape()).contiguous()
    n = int(round(cfg["t_end"] / cfg["dt"]))
    t = R.rbffd_step(ctx, model, s, 0.0, cfg["dt"], n, R.RK4)
    assert abs(t - 900.0) < 1e-9
    R.rbffd_ghost(ctx, model, s)
    return cfg, s.double().cpu().numpy().reshape(-1, 4)


def test_density_current_converges():
    """Section 6.4 (convergence of the density current): Cartesian nodes at
    400, 200, 100 and 50 m against a 25 m run of the same method on nested
    nodes, theta' at t = 900 s compared on the 400 m nodes; the paper reports
    third-order convergence of theta' for h <= 200 m: here every halving
    below 200 m is above order 2.3 and their mean above 2.8."""
    ref_cfg, ref_y = run_density_current("cartesian", 25.0)
    hs = (400.0, 200.0, 100.0, 50.0)
    runs = [run_density_current("cartesian", h) for h in hs]
    errs = _shared_errors(ref_cfg, ref_y, runs, 400.0)
    orders = [np.log2(errs[k] / errs[k + 1]) for k in range(len(hs) - 1)]
    print(f"   theta' rel-l2 vs 25 m at {hs} m: {['%.2e' % e for e in errs]}, "
          f"orders {['%.2f' % o for o in orders]}", flush=True)
    # measured: errors 0.474, 0.402, 0.0669, 0.00408; orders 0.24, 2.59, 4.04 (3.3 on
    # average from 200 m to 50 m; the 400 m grid does not resolve the current)
    assert all(errs[k + 1] < errs[k] for k in range(len(hs) - 1))
    assert min(orders[1:]) > 2.3 and np.log2(errs[1] / errs[3]) / 2 > 2.8


def test_density_current_25m_fp64_fp32_bf16_to_900s():
    """The 2048 x 256 channel (25 m columns, 524,288 nodes) run to t = 900 s
    (14,400 RK4 steps) in FP64, FP32 and with BF16 weights. FP64 against the
    25 m reference row of Table tbl:straka (extrema within 0.5% / 0.05 K,
    front within 0.2%); FP32 within 1e-4 theta' rel-l2 of FP64 (measured
    7e-6); BF16 weights within 0.1 (measured 0.033)."""
    import torch
    from paper_1509_02615_amd import rbffd as R
    from paper_1509_02615_amd import pipeline as P
    from workloads import scale_config
    print("density current 2048x256 to 900 s: FP64, FP32, BF16 weights", flush=True)
    ctx = R.Context(0)
    cfg = scale_config()
    nd = cfg["nodes"]
    xy, idx, W, Ww, (sa, sw) = P.ns_weights(ctx, cfg)
    assert int(sa.abs().sum()) == 0 and int(sw.abs().sum()) == 0
    th = {}
    for name, (fdt, wdt) in {"fp64": (0, 0), "fp32": (1, 1), "bf16": (1, 2)}.items():
        model = P.ns_model(ctx, cfg, idx, W, Ww, xy=xy, field_dtype=fdt, weight_dtype=wdt)
        s = P.to_dev(cfg["state0"], torch.float64 if fdt == 0 else torch.float32).reshape(model.state_shape()).contiguous()
        t = 0.0
        for _ in range(8):
            t = R.rbffd_step(ctx, model, s, t, cfg["dt"], 1800, R.RK4)
        assert abs(t - 900.0) < 1e-9
        R.rbffd_ghost(ctx, model, s)
        y = s.double().cpu().numpy().reshape(-1, 4)
        th[name] = y[:nd.n_active, 2]
        if name == "fp64":
            e = O.extrema(y, nd.n_active)
            front = O.front_location(nd.xy, y[:, 2], nd.wall_nodes[0])
            got = [e["theta_min"], e["theta_max"], e["w_min"], e["w_max"], front]
            ref = table_row("reference", 25.0)
            print(f"   fp64: got {np.round(got, 3).tolist()} table (25 m reference) {ref}", flush=True)
            for g, r in zip(got[:4], ref[:4]):
                assert abs(g - r) <= 0.005 * abs(r) + 0.05, (got, ref)
            assert abs(front - ref[4]) <= 0.002 * ref[4]
        del model
    r32 = np.linalg.norm(th["fp32"] - th["fp64"]) / np.linalg.norm(th["fp64"])
    rbf = np.linalg.norm(th["bf16"] - th["fp64"]) / np.linalg.norm(th["fp64"])
    print(f"   theta' rel-l2 vs FP64 at 900 s: FP32 {r32:.2e}, BF16 weights {rbf:.2e}", flush=True)
    assert r32 <= 1e-4 and rbf <= 0.1
