"""Benchmark of the RBF-FD hot path on one MI355X.

Workload: the density current on a 2048 x 256 hexagonal-row channel at 25 m
column spacing (524,288 active nodes + 2 x 2,048 ghost nodes), r^7 +
degree-4 polynomials, n = 37, operators Dx, Dz, Lap, Lap^3, RK4 with
dt = 1/16 s. Setup (untimed for the headline, reported separately): stencil
search + batched weights (A1-A4) and model creation. Timed region: K RK4
steps, each 4 stages of ghost closure (B1) + fused gather-stencil RHS and
stage update (B2-B4), with HIP events around every fused RHS launch.

    python bench.py [--steps K] [--warmup W] [--precision fp32|fp64|bf16]

Prints one JSON line. value = node updates per second (one node, one RHS
evaluation) of the FP32-field path; roofline = the fused RHS kernel's
algorithmic bytes per launch over its measured average duration.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
FP64_PEAK_TFLOPS = 78.6
# closure network per node-sample: 149 inputs -> 128 -> 128 -> 4 outputs,
# 2 flops per multiply-add (the kernels pad to 160 inputs and 16 outputs)
CLOSURE_FLOP_PER_SAMPLE = 2 * (149 * 128 + 128 * 128 + 128 * 4)
ROOT = os.path.dirname(os.path.abspath(__file__))
COUNTERS = os.path.join(ROOT, "profiles", "ns_stage_kernel_hbm_counters.json")
# Fixed algorithmic bytes per node-update of one RHS evaluation (all four
# fields read and written once, int32 indices, 37 slots): FP32 Dx, Dz, Lap +
# FP64 Lap^k weights 920 B; FP64 everything 1,396 B; BF16 Dx, Dz, Lap + FP64
# Lap^k 698 B. The kernels stream fewer bytes (16-bit offsets, the centre slot
# left out, Lap^k as FP32 + correction); `frac` uses their own count, and
# `frac_fixed_count` this fixed one.
FIXED_BYTES_PER_NODE = {"fp32": 920.0, "fp64": 1396.0, "bf16": 698.0}
METRIC = "RHS node-updates/s & % HBM peak, FP32 vs FP64 at stated rel-L2; stencils/s"


def field_bytes_per_node_stage(tableau, fb, F=4, E=1):
    """Field traffic per node and stage, averaged over the tableau's stages:
    RK4 stage 1 reads y_n and writes y_1 and the accumulator; stages 2-3 read
    y_s, y_n and the accumulator and write y_s+1 and the accumulator;
    stage 4 reads y_3 and the accumulator and writes y_n+1."""
    v = F * E * fb
    if tableau == "rk4":
        return v * (3 + 5 + 5 + 3) / 4.0
    return v * (2 + 3 + 3) / 3.0


def measured_traffic(leg, bytes_per_launch):
    """HBM bytes per launch (GB) of the stage kernel of one bench leg (fp32,
    fp64, bf16, ensemble64_fp32_row, ensemble64_fp32_morton) from the
    committed counter passes, if the kernel sources still hash as when
    counted and the algorithmic count is the same."""
    import hashlib
    try:
        d = json.load(open(COUNTERS))
        src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in d["sources"])
        rec = d["legs"][leg]
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != d["source_sha256"]:
        return None
    if abs(rec["algorithmic_bytes_per_launch"] - bytes_per_launch) > 1.0:
        return None
    return rec["traffic_bytes_per_launch"] / 1e9          # GB per launch, like `achieved` per second


def leg_roofline(leg, res, n_active):
    """Roofline of one stage-kernel leg: algorithmic bytes per launch (the
    kernel's own count, and the fixed count where one is defined) over the
    HIP-event average launch duration, against the 8 TB/s HBM peak, with the
    counter-measured traffic where committed."""
    k_s = res["kernel_avg_ms"] / 1e3
    counted = leg
    if leg.startswith("ensemble"):   # the traversal the tuner kept: shapes 6-11 are Morton order
        counted = f"{leg}_{'morton' if res.get('tuned_shape', 0) >= 6 else 'row'}"
    out = {"bound": "hbm", "achieved": res["bytes_per_launch"] / k_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": res["bytes_per_launch"] / k_s / 1e9 / HBM_PEAK_GBS,
           "traffic": measured_traffic(counted, res["bytes_per_launch"]),
           "traffic_unit": "GB per launch (HBM counters, calibrated)", "kernel": "ns_stage_kernel",
           "bytes_per_launch": res["bytes_per_launch"], "kernel_avg_ms": res["kernel_avg_ms"]}
    fixed = FIXED_BYTES_PER_NODE.get(leg)
    if fixed is not None:
        out["fixed_bytes_per_node"] = fixed
        out["frac_fixed_count"] = fixed * n_active / k_s / 1e9 / HBM_PEAK_GBS
    return out


def run_rhs_leg(R, P, ctx, cfg, idx, W, Ww, xy, fdt, wdt, steps, warmup, ensemble=1):
    import torch
    nd = cfg["nodes"]
    model = P.ns_model(ctx, cfg, idx, W, Ww, xy=xy, field_dtype=fdt, weight_dtype=wdt, ensemble=ensemble)
    dt_t = torch.float64 if fdt == R.F64 else torch.float32
    s0 = np.repeat(cfg["state0"][:, None, :], ensemble, axis=1)
    if ensemble > 1:   # members differ in the bubble amplitude, U[-17, -13] K
        from workloads.fields import ensemble_amplitudes
        s0 = s0 * (ensemble_amplitudes(ensemble) / -15.0)[None, :, None]
    state = P.to_dev(s0, dt_t).reshape(model.state_shape()).contiguous()
    shape, tune_us = R.rbffd_model_tune(ctx, model, state)
    t = R.rbffd_step(ctx, model, state, 0.0, cfg["dt"], warmup, R.RK4)   # warm-up
    # set-up outside the timed region: rbffd_step captures its eight-step and
    # one-step graphs when a call first needs them, so eight more steps from a
    # saved copy capture the first; the state then goes back to the copy (the
    # graphs are bound to this buffer, not to its contents)
    saved = state.clone()
    R.rbffd_step(ctx, model, state, t, cfg["dt"], 8 + (1 if warmup % 8 == 0 else 0), R.RK4)
    state.copy_(saved)
    del saved
    # timed region: K steps, each one replay of the captured step graph
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record()
    t = R.rbffd_step(ctx, model, state, t, cfg["dt"], steps, R.RK4)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    total_ms = ev0.elapsed_time(ev1)
    # kernel durations (outside the timed region): K more steps launched one
    # stage at a time with HIP events around every fused RHS launch
    model.profile(True)
    model.profile_read()
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    t = R.rbffd_step(ctx, model, state, t, cfg["dt"], steps, R.RK4)
    torch.cuda.synchronize()
    prof_s = time.perf_counter() - p0
    k_ms, launches = model.profile_read()
    model.profile(False)
    fb = 8 if fdt == R.F64 else 4
    per_node = model.bytes_per_node() + field_bytes_per_node_stage("rk4", fb, E=ensemble)
    bytes_launch = per_node * nd.n_active
    k_avg_s = k_ms / launches / 1e3
    updates = nd.n_active * ensemble * 4 * steps
    res = dict(node_updates_per_s=updates / (total_ms / 1e3), ms_per_step=total_ms / steps,
               wall_s=wall, profiled_ms_per_step=prof_s * 1e3 / steps,
               kernel_avg_ms=k_ms / launches, kernel_launches=launches,
               bytes_per_node=per_node, bytes_per_launch=bytes_launch,
               kernel_gbs=bytes_launch / k_avg_s / 1e9,
               finite=bool(torch.isfinite(state).all().item()), tuned_shape=shape, tune_us=tune_us)
    if ensemble > 1:
        # 36 streamed slots (the centre's adds an exact zero and is left out) x (4 differences
        # + 15 multiply-adds) + ~60 epilogue flops per member-node, counted as 2 per
        # multiply-add. With 64k members every sum is FP64: the FP64 vector rate equals
        # the FP32 one without packed instructions (78.6 TFLOP/s)
        flops = nd.n_active * ensemble * (36 * (4 + 2 * 15) + 60)
        res["kernel_tflops"] = flops / k_avg_s / 1e12
        res["valu_frac_fp64_peak"] = res["kernel_tflops"] / FP64_PEAK_TFLOPS
        res["valu_frac_fp32_peak"] = res["kernel_tflops"] / FP32_VALU_PEAK_TFLOPS
    del model
    return res


def weights_leg(R, ctx, cfg, precision, ref=None):
    """One rbffd_weights call over a node set, after an untimed one; returns
    stencils/s (and, given the oracle's weights of sampled stencils, the
    worst sampled error)."""
    import torch
    from paper_1509_02615_amd import pipeline as P
    nd = cfg["nodes"]
    xy = P.to_dev(nd.xy, torch.float64)
    n_per = P.to_dev(cfg["n_per"], torch.int32)
    m_per = P.to_dev(cfg["m_per"], torch.int32)
    l_per = P.to_dev(cfg["l_per"], torch.int32)
    ops = [(R.DX, 0, 0), (R.DZ, 0, 0), (R.HYPERLAP, 0, 0)]
    idx = R.rbffd_knn(ctx, xy, cfg["n_max"], 0.0, n_per=n_per)
    # one untimed tuning call first (each size bucket's launch shape, kept in
    # the context); the timed call then also finds its output blocks (1.5 GB
    # of weights) in torch's allocator, as a steady-state caller would
    t0 = time.perf_counter()
    _, W, _, _, shapes, bucket_ms = R.rbffd_weights_tune(ctx, xy, ops, cfg["n_max"], n_per=n_per, m_per=m_per,
                                                         l_per=l_per, idx_in=idx, precision=precision)
    tune_s = time.perf_counter() - t0
    del W
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    _, W, status, rc = R.rbffd_weights(ctx, xy, ops, cfg["n_max"], n_per=n_per, m_per=m_per, l_per=l_per,
                                       idx_in=idx, precision=precision)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    bad = int(((status == 1) | (status == 2)).sum().item())
    fallback = int((status == 3).sum().item())   # solved again in FP64 (FP32 factorisation only)
    err = None
    if ref:
        rows = torch.tensor(sorted(ref), device=W.device)
        err = sampled_weights_error(idx[rows].cpu().numpy(), W[:, rows].cpu().numpy(), ref)
    # algorithmic flops of the solves: LU of K x K (2/3 K^3) and the forward and
    # back substitution of the 3 right-hand sides (2 K^2 each); K = n + M
    K = cfg["n_per"].astype(np.float64) + (cfg["l_per"] + 1) * (cfg["l_per"] + 2) / 2
    flops = float(np.sum(2.0 / 3.0 * K ** 3 + 2.0 * K ** 2 * 3))
    return dict(stencils=nd.n_active, ms=ms, stencils_per_s=nd.n_active / (ms / 1e3), singular=bad,
                fp64_fallback=fallback, sampled_worst_rel_err_vs_oracle=err,
                tuned_shapes=shapes, tuned_bucket_ms=bucket_ms, tune_s=tune_s,
                sampled=None if not ref else f"{len(ref)} stencils (every 997th centre)",
                solve_tflops=flops / (ms / 1e3) / 1e12,
                fp64_peak_frac=flops / (ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
                note="solve flops only (2/3 K^3 + 2 K^2 per right-hand side); assembly and "
                     "double-double refinement are extra work, not counted")


def advection_leg(R, P, ctx):
    """The scalar-transport workload (64 x 64 Cartesian nodes on the unit
    square, r^5 + degree-4 polynomials, Dx, Dy and Lap^3, FP64): search and
    weights, then the whole RK4 run to T = 5 (2,000 steps, one captured graph
    per step) and the bell-return error against the initial field, which is
    the exact solution at T. The 4,096-node state is cache-resident, so the
    run measures per-step launch cost rather than bandwidth."""
    import numpy as np
    import torch
    from workloads import advection_config
    cfg = advection_config(64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xy, idx, W, status = P.advection_weights(ctx, cfg)
    model = P.advection_model(ctx, cfg, idx, W, xy=xy)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    psi0 = cfg["psi0"]
    n = int(round(cfg["t_end"] / cfg["dt"]))
    s = P.to_dev(psi0, torch.float64).reshape(model.state_shape()).contiguous()
    s0 = s.clone()
    R.rbffd_step(ctx, model, s, 0.0, cfg["dt"], 20, R.RK4)   # capture and warm up on the same buffer
    s.copy_(s0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = R.rbffd_step(ctx, model, s, 0.0, cfg["dt"], n, R.RK4)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    y = s.double().cpu().numpy().ravel()
    return dict(nodes=int(cfg["nodes"].n_active), steps=n, t_end=float(t), setup_s=setup, run_s=sec,
                us_per_step=sec / n * 1e6, rhs_per_s=4 * n / sec, singular=int(status.abs().sum()),
                bell_return_rel_l2=float(np.linalg.norm(y - psi0) / np.linalg.norm(psi0)),
                bell_return_max_abs=float(np.abs(y - psi0).max()))


def fullrun_leg(R, P, ctx, cfg, idx, W, Ww, xy, t_end=900.0, chunk=1800):
    """The density current on the 2048 x 256 channel run to t_end with FP64,
    FP32 and BF16-weight fields/weights from the same initial state (RK4,
    dt = 1/16 s, 14,400 steps): theta' rel-l2 over the active nodes of the
    reduced-precision runs against the FP64 run, and each run's theta'/w'
    extrema and front (the -0.5 K contour on the ground)."""
    import torch
    nd = cfg["nodes"]
    n = int(round(t_end / cfg["dt"]))
    out, fields = {}, {}
    for name, (fdt, wdt) in {"fp64": (R.F64, R.F64), "fp32": (R.F32, R.F32), "bf16": (R.F32, R.BF16)}.items():
        model = P.ns_model(ctx, cfg, idx, W, Ww, xy=xy, field_dtype=fdt, weight_dtype=wdt)
        s = P.to_dev(cfg["state0"], torch.float64 if fdt == R.F64 else torch.float32)
        s = s.reshape(model.state_shape()).contiguous()
        t, done = 0.0, 0
        w0 = time.perf_counter()
        while done < n:
            k = min(chunk, n - done)
            t = R.rbffd_step(ctx, model, s, t, cfg["dt"], k, R.RK4)
            done += k
        R.rbffd_ghost(ctx, model, s)
        torch.cuda.synchronize()
        y = s.double().cpu().numpy().reshape(-1, 4)
        na = nd.n_active
        th = y[:na, 2]
        bottom = nd.wall_nodes[0]
        x, tb = nd.xy[bottom, 0], y[bottom, 2]
        cold = np.nonzero((tb <= -0.5) & (x >= 0.0))[0]
        front = None
        if cold.size:
            i = cold[np.argmax(x[cold])]
            j = i + 1 if i + 1 < bottom.size else i
            front = float(x[i] + (-0.5 - tb[i]) / (tb[j] - tb[i]) * (x[j] - x[i])) if j != i and tb[j] != tb[i] else float(x[i])
        fields[name] = th
        out[name] = dict(seconds=time.perf_counter() - w0, steps=n, t=t, theta_min=float(th.min()),
                         theta_max=float(th.max()), w_min=float(y[:na, 1].min()), w_max=float(y[:na, 1].max()),
                         front_m=front)
        del model
    ref = fields["fp64"]
    for name in ("fp32", "bf16"):
        out[name]["theta_rel_l2_vs_fp64"] = float(np.linalg.norm(fields[name] - ref) / np.linalg.norm(ref))
    return out


def device_peaks_leg(R, ctx):
    """The device's practical ceilings beside the published peaks: a plain
    streaming copy of 512 MiB (read + write bytes per second) and the
    matrix-core probe (dense BF16 16x16x32 products on registers)."""
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    src = torch.ones(512 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    R.rbffd_stream_copy(ctx, dst, src)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(5):
        R.rbffd_stream_copy(ctx, dst, src)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() / (ev0.elapsed_time(ev1) / 1e3) / 1e9
    del src, dst
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    out = torch.empty(1024 * n_cu, dtype=torch.float32, device="cuda")
    res = dict(stream_copy_512MiB_gbs=copy_gbs, stream_copy_frac_of_peak=copy_gbs / HBM_PEAK_GBS)
    for shape, name in ((0, "16x16x32"), (1, "32x32x16")):
        R.rbffd_mfma_probe(ctx, out, 100, shape)
        torch.cuda.synchronize()
        ev0.record()
        flops = R.rbffd_mfma_probe(ctx, out, 20000, shape)
        ev1.record()
        torch.cuda.synchronize()
        tf = flops / (ev0.elapsed_time(ev1) / 1e3) / 1e12
        res[f"mfma_bf16_{name}_tflops"] = tf
        res[f"mfma_bf16_{name}_frac_of_peak"] = tf / BF16_MFMA_PEAK_TFLOPS
    return res


def closure_leg(R, ctx, calls=20, members=256):
    """Learned closure on its coarse grid (400 m Cartesian channel, 128 x 17
    nodes) for 256 members: 557,056 node-samples per fused forward call
    (relu network, seeded random weights, a state developed by 60 plain
    steps), timed over `calls` calls; plus the corrected coarse step against
    the plain one."""
    import torch
    from paper_1509_02615_amd import closure as CL
    from workloads import closure_config
    from workloads.fields import ensemble_amplitudes
    cc = closure_config()
    cm, _ = CL.coarse_model(ctx, cc, members)
    dt = cc["coarse"]["dt"]
    state = CL.to_full(cm, CL.ensemble_state(cc["coarse"], ensemble_amplitudes(members))[:cm.Na])
    R.rbffd_step(ctx, cm, state, 0.0, dt, 60, R.RK4)
    rng = np.random.default_rng(7)
    blocks = [rng.uniform(-1, 1, (128, 160)) / np.sqrt(149.0), rng.normal(0, 0.1, 128),
              rng.uniform(-1, 1, (128, 128)) / np.sqrt(128.0), rng.normal(0, 0.1, 128),
              np.vstack([rng.uniform(-1, 1, (4, 128)) / np.sqrt(128.0), np.zeros((12, 128))]),
              np.concatenate([rng.normal(0, 0.1, 4), np.zeros(12)])]
    params = torch.from_numpy(np.concatenate([b.ravel() for b in blocks]).astype(np.float32)).cuda()
    nodef = torch.from_numpy(cc["node_feature"]).cuda()
    cl = R.Closure(ctx, cm, params, nodef, [2.0, 2.0, 1.8, 3e-4], [1e-3, 1e-3, 7e-4, 3e-6],
                   activation=R.ACT_RELU)
    S = cm.Na * members
    R.rbffd_model_tune(ctx, cm, state)    # the coarse steps in their tuned launch shape
    shape, tune_us = cl.tune(state)
    for _ in range(3):
        cl.forward(state)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(calls):
        cl.forward(state)
    ev1.record()
    torch.cuda.synchronize()
    fwd_s = ev0.elapsed_time(ev1) / calls / 1e3
    tflops = S * CLOSURE_FLOP_PER_SAMPLE / fwd_s / 1e12
    n = 10
    ev0.record()
    R.rbffd_step(ctx, cm, state, 0.0, dt, n, R.RK4)
    ev1.record()
    torch.cuda.synchronize()
    plain_ms = ev0.elapsed_time(ev1) / n
    ev0.record()
    cl.step(state, 0.0, dt, n, R.RK4)
    ev1.record()
    torch.cuda.synchronize()
    corr_ms = ev0.elapsed_time(ev1) / n
    speedup = closure_speedup(R, ctx, cc, params, nodef)
    return dict(samples=S, forward_us=fwd_s * 1e6, samples_per_s=S / fwd_s, tuned_shape=shape, tune_us=tune_us,
                roofline={"bound": "mfma", "achieved": tflops, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": tflops / BF16_MFMA_PEAK_TFLOPS, "flop_per_sample": CLOSURE_FLOP_PER_SAMPLE},
                plain_step_ms=plain_ms, corrected_step_ms=corr_ms, vs_fine_run=speedup,
                note="forward call = fused gather + 3-layer network kernel + output scaling; "
                     "steps: 4-stage RK4 of 256 members, corrected = plain + forward + correction")


def closure_quality_leg(R, ctx, members=256, n_train=192):
    """The learned closure's quality at the workload's 256 members: fine
    (50 m) snapshots over 150 s, one-step targets, training on 192 members,
    plain and corrected coarse (400 m) runs of the 64 held-out members,
    theta' relative l2 against their fine runs at 30, 60, 120 and 150 s."""
    from paper_1509_02615_amd import closure as CL
    from workloads import closure_config
    q = CL.quality_run(ctx, closure_config(n_members=members, n_train=n_train))
    q["errors"] = {str(c): {"plain": e[0], "corrected": e[1]} for c, e in q["errors"].items()}
    return q


def closure_speedup(R, ctx, cc, params, nodef, members=64, seconds=30.0):
    """Cost of the corrected coarse run against the fine run it stands in
    for: the same members and the same simulated interval (30 s), each on
    its own grid (fine 50 m, 1024 x 129 nodes, dt = 1/8 s; coarse 400 m,
    128 x 17, dt = 1 s), timed after a warm-up that captures the graphs."""
    import torch
    from paper_1509_02615_amd import closure as CL
    from paper_1509_02615_amd import pipeline as P
    from workloads.fields import ensemble_amplitudes
    amps = ensemble_amplitudes(members)
    fine = cc["fine"]
    xy, idx, W, Ww, _ = P.ns_weights(ctx, fine)
    fm = P.ns_model(ctx, fine, idx, W, Ww, xy=xy, field_dtype=R.F32, weight_dtype=R.F32, ensemble=members)
    fs = CL.ensemble_state(fine, amps)
    cm, _ = CL.coarse_model(ctx, cc, members)
    cs = CL.to_full(cm, CL.ensemble_state(cc["coarse"], amps)[:cm.Na])
    cl = R.Closure(ctx, cm, params, nodef, [2.0, 2.0, 1.8, 3e-4], [1e-3, 1e-3, 7e-4, 3e-6], activation=R.ACT_RELU)
    # both runs in their tuned launch shapes
    fine_shape, _ = R.rbffd_model_tune(ctx, fm, fs)
    coarse_shape, _ = R.rbffd_model_tune(ctx, cm, cs)
    cl.tune(cs)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    nf = int(round(seconds / fine["dt"]))
    nc = int(round(seconds / cc["coarse"]["dt"]))
    f0, c0 = fs.clone(), cs.clone()
    R.rbffd_step(ctx, fm, fs, 0.0, fine["dt"], 8, R.RK4)       # graph capture, warm-up
    cl.step(cs, 0.0, cc["coarse"]["dt"], 4, R.RK4)
    R.rbffd_step(ctx, cm, cs, 0.0, cc["coarse"]["dt"], 4, R.RK4)
    fs.copy_(f0)
    cs.copy_(c0)
    fine_s = timed(lambda: R.rbffd_step(ctx, fm, fs, 0.0, fine["dt"], nf, R.RK4))
    corr_s = timed(lambda: cl.step(cs, 0.0, cc["coarse"]["dt"], nc, R.RK4))
    cs.copy_(c0)
    plain_s = timed(lambda: R.rbffd_step(ctx, cm, cs, 0.0, cc["coarse"]["dt"], nc, R.RK4))
    return dict(members=members, simulated_s=seconds, fine_steps=nf, coarse_steps=nc, fine_run_s=fine_s,
                corrected_run_s=corr_s, plain_coarse_run_s=plain_s, speedup_corrected_vs_fine=fine_s / corr_s,
                fine_shape=fine_shape, coarse_shape=coarse_shape)


def cpu_oracle_weights(min_seconds=10.0):
    """The oracle's weights (extended-precision assembly, LU, refinement) on a
    bounded sample of the mixed 1M batch: 120 stencils (every 997th centre;
    their stencils found by the oracle's search beforehand, untimed), solved
    repeatedly until min_seconds have passed, on one thread and then in one
    process per core. The solves see only the sample's nodes (renumbered), so
    that no call converts all 1M coordinates. Also returns the sample's
    oracle stencils and weights, against which the GPU weights legs report
    their accuracy."""
    import oracle as O
    from workloads import weights_config
    cfg = weights_config(1024)
    nd = cfg["nodes"]
    sample = np.arange(0, nd.n_active, 997)[:120]
    stencils = [O.knn(nd.xy, [c], int(cfg["n_per"][c]), 0.0)[0] for c in sample]
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.HYPERLAP, 0, 0)]
    used = np.unique(np.concatenate([sample] + stencils))
    local = lambda a: np.searchsorted(used, a)
    job = (nd.xy[used], [(local(st), int(local(c)), int(cfg["m_per"][c]), int(cfg["l_per"][c]))
                         for c, st in zip(sample, stencils)], ops)
    ref = {int(c): (st, O.stencil_weights(*_solve_args(job, a))[0])
           for a, (c, st) in enumerate(zip(sample, stencils))}
    done, el = _oracle_weights_worker((job, min_seconds))
    res = dict(value=done / el, unit="stencils/s", cores=1, kind="oracle", host=host_cpu(),
               sample=f"{done} solves of 120 stencils of the mixed 1M batch (every 997th centre), "
                      f"{el:.1f} s (numpy/scipy, single thread)")
    res["all_cores"] = _all_cores(_oracle_weights_worker, job, min_seconds, 1, "stencils/s",
                                  "the same 120 stencils")
    return res, ref


def _solve_args(job, a):
    """Arguments of the oracle's stencil_weights for stencil a of a job."""
    xy, stencils, ops = job
    st, c, m, l = stencils[a]
    return xy, st, c, m, l, ops, 0.0


def _oracle_weights_worker(args):
    """One worker process of the all-cores weights baseline: the sample's
    stencils solved by the oracle in turn for `seconds`; returns the number
    of solves and the time taken."""
    job, seconds = args
    import oracle as O
    with one_thread():
        done, t0 = 0, time.perf_counter()
        while True:
            for a in range(len(job[1])):
                O.stencil_weights(*_solve_args(job, a))
                done += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                return done, el


def one_thread():
    """Limits the BLAS/OpenMP pools of numpy and scipy to one thread, so an
    oracle timing uses the cores it reports."""
    from threadpoolctl import threadpool_limits
    return threadpool_limits(1)


def host_cpu():
    """The host processor's model name and the cores this process may use."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name} ({len(os.sched_getaffinity(0))} cores available)"


def sampled_weights_error(idx, W, ref):
    """Worst norm-wise relative error, per stencil and operator, of GPU
    weights against the oracle's at the sampled centres: idx [S][n_max] and
    W [ops][S][n_max] hold the GPU rows of the centres in sorted order (None
    when a sampled stencil differs)."""
    worst = 0.0
    for a, c in enumerate(sorted(ref)):
        st, Wo = ref[c]
        n = len(st)
        if not np.array_equal(idx[a, :n], st):
            return None
        for o in range(Wo.shape[0]):
            worst = max(worst, float(np.linalg.norm(W[o, a, :n] - Wo[o]) / np.linalg.norm(Wo[o])))
    return worst


def cpu_baseline(cfg, min_seconds=10.0):
    """The oracle's RHS on a bounded sample: one 2048-node row of the same
    channel (row 128), stencils and weights from the oracle (untimed), then
    repeated evaluations of Eqs. uEq..piEq for at least min_seconds. The
    evaluation is the oracle's own full-model path (ns_rhs): the four
    differentiation matrices as sparse products (the sample rows' DMs, built
    untimed), then the pointwise physics."""
    import oracle as O
    nd = cfg["nodes"]
    rows = np.arange(128 * nd.nx, 129 * nd.nx)
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.LAP, 0, 0), (O.HYPERLAP, 3, 7)]
    idx = O.knn(nd.xy, rows, cfg["n"], nd.period_x)
    Wo, _ = O.all_weights(nd.xy, idx, rows, cfg["m"], cfg["l"], ops, nd.period_x)
    state = cfg["state0"].astype(np.float64)
    D = [O.dm_matrix(idx, W, state.shape[0]) for W in Wo]
    is_wall = np.zeros(len(rows), bool)
    job = (state, rows, idx, Wo, D, nd.xy[rows, 1], is_wall, cfg["consts"], cfg["hv_coeff"])
    reps, el = _oracle_rhs_worker((job, min_seconds))
    res = dict(value=len(rows) * reps / el, unit="node-updates/s", cores=1, kind="oracle", host=host_cpu(),
               sample=f"one 2048-node row of the 2048x256 channel, {reps} FP64 RHS evaluations "
                      f"in {el:.1f} s (numpy and scipy sparse products, single thread)")
    res["all_cores"] = _all_cores(_oracle_rhs_worker, job, min_seconds, len(rows), "node-updates/s",
                                  "the same row")
    return res


def _oracle_rhs_worker(args):
    """The oracle RHS on the sample row (sparse products of the four
    differentiation matrices, then Eqs. uEq..piEq), repeated for `seconds`
    on one thread; returns the number of evaluations and the time taken.
    Also one worker process of the all-cores baseline."""
    (state, rows, idx, Wo, D, z, is_wall, consts, hv), seconds = args
    import oracle as O
    with one_thread():
        reps, t0 = 0, time.perf_counter()
        while True:
            O.ns_tendency(state, rows, idx, Wo[0], Wo[1], Wo[2], Wo[3], z, is_wall, consts, hv,
                          derivs=[Dm @ state for Dm in D])
            reps += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                return reps, el


def _all_cores(worker, job, seconds, units_per_rep, unit, what):
    """An oracle worker on every host core it may use (at most 16): one
    process each, started fresh (they never touch the GPU), all timed
    together; `units_per_rep` converts a worker's repetitions to `unit`."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    try:
        with ProcessPoolExecutor(cores, mp_context=mp.get_context("spawn")) as ex:
            # a first round starts the workers (imports), the second is timed
            list(ex.map(worker, [(job, 0.0)] * cores, timeout=300))
            done = list(ex.map(worker, [(job, seconds)] * cores, timeout=seconds + 300))
    except Exception as exc:  # a broken or slow pool leaves the single-thread figure alone
        print(f"[bench] all-cores oracle baseline skipped: {exc!r}", file=sys.stderr, flush=True)
        return None
    # each process times its own loop; the processes run at the same time
    rate = sum(units_per_rep * reps / el for reps, el in done)
    return dict(value=rate, unit=unit, cores=cores, kind="oracle",
                sample=f"{what} in {cores} processes at once, {sum(r for r, _ in done)} repetitions "
                       f"over {max(el for _, el in done):.1f} s each")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the other precisions and weight legs")
    ap.add_argument("--closure-only", action="store_true",
                    help="run only the learned-closure leg and print its result (for profiling)")
    ap.add_argument("--weights-only", action="store_true",
                    help="run only the mixed 1M-stencil weights batch once (after one tuning call) and print "
                         "its result (for profiling)")
    ap.add_argument("--weights-precision", default="fp64", choices=["fp64", "fp32_ir"],
                    help="solve precision of --weights-only: FP64, or the FP32 factorisation with FP64 "
                         "refinement")
    ap.add_argument("--fullrun-only", action="store_true",
                    help="run only the FP64/FP32/BF16 runs to t = 900 s and print their comparison")
    ap.add_argument("--pmc-run", action="store_true",
                    help="short run for hardware-counter passes: 2 RK4 steps of the chosen precision "
                         "(and --ensemble) and 3 plain copies of 512 MiB (counter calibration); prints no "
                         "JSON line")
    ap.add_argument("--ensemble", type=int, default=1, help="members of the --pmc-run model")
    ap.add_argument("--shape", type=int, default=-1,
                    help="stage-kernel launch shape of the --pmc-run model (-1: tuned; with 64 members "
                         "6-11 are 0-5 in Morton order)")
    ap.add_argument("--no-fullrun", action="store_true", help="skip the runs to t = 900 s (for profiling)")
    ap.add_argument("--no-closure-quality", action="store_true",
                    help="skip the 256-member closure training and held-out comparison (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the multi-GPU path is not built (see the sharding notes); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # The oracle baselines run first, on the host alone: their worker
    # processes start before this process touches the GPU.
    cpu, cpu_weights, oracle_ref = None, None, None
    if not (args.no_cpu_baseline or args.closure_only or args.weights_only or args.fullrun_only or args.pmc_run):
        from workloads import scale_config as _scale
        cpu = cpu_baseline(_scale())
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)
        if not args.no_extras:
            cpu_weights, oracle_ref = cpu_oracle_weights()
            print(f"[bench] cpu oracle weights: {cpu_weights}", file=sys.stderr, flush=True)

    import torch
    from paper_1509_02615_amd import rbffd as R
    from paper_1509_02615_amd import pipeline as P
    from workloads import scale_config, weights_config

    torch.cuda.set_device(0)
    ctx = R.Context(0)
    if args.closure_only:
        print(json.dumps(closure_leg(R, ctx, calls=args.steps)), flush=True)
        return
    if args.weights_only:
        from workloads import weights_config
        prec = R.SOLVE_FP64 if args.weights_precision == "fp64" else R.SOLVE_FP32_IR
        print(json.dumps(weights_leg(R, ctx, weights_config(1024), prec)), flush=True)
        return
    cfg = scale_config()
    nd = cfg["nodes"]
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    log(f"[bench] workload {cfg['name']}: {nd.n_active} active + {nd.n_total - nd.n_active} ghost nodes")

    # A1-A4 on the same node set (setup of the timed region)
    xy = P.to_dev(nd.xy, torch.float64)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    xy, idx, W, Ww, (st_a, st_w) = P.ns_weights(ctx, cfg, xy=xy)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - s0
    n_stencils = nd.n_active + nd.bnd_nodes.size
    assert int(st_a.abs().sum()) == 0 and int(st_w.abs().sum()) == 0
    log(f"[bench] search + weights for {n_stencils} stencils: {setup_s:.3f} s")
    if args.fullrun_only:
        print(json.dumps(fullrun_leg(R, P, ctx, cfg, idx, W, Ww, xy)), flush=True)
        return

    fdt = {"fp32": R.F32, "fp64": R.F64, "bf16": R.F32}[args.precision]
    wdt = {"fp32": R.F32, "fp64": R.F64, "bf16": R.BF16}[args.precision]
    if args.pmc_run:
        E = args.ensemble
        model = P.ns_model(ctx, cfg, idx, W, Ww, xy=xy, field_dtype=fdt, weight_dtype=wdt, ensemble=E)
        s0 = np.repeat(cfg["state0"][:, None, :], E, axis=1)
        state = P.to_dev(s0, torch.float64 if fdt == R.F64 else torch.float32)
        state = state.reshape(model.state_shape()).contiguous()
        shape, _ = R.rbffd_model_tune(ctx, model, state, args.shape)   # as in the timed region unless forced
        R.rbffd_step(ctx, model, state, 0.0, cfg["dt"], 2, R.RK4)
        src = torch.ones(512 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            R.rbffd_stream_copy(ctx, dst, src)
        torch.cuda.synchronize()
        log(f"[bench] pmc run done: E = {E}, stage kernel shape {shape}, {model.bytes_per_node()} B/node stencil "
            f"stream, copy kernel 2 x {512 << 20} bytes per launch")
        return
    main_leg = run_rhs_leg(R, P, ctx, cfg, idx, W, Ww, xy, fdt, wdt, args.steps, args.warmup)
    log(f"[bench] {args.precision}: {main_leg}")

    extras = {}
    if not args.no_extras:
        for name, (f2, w2) in {"fp64": (R.F64, R.F64), "fp32": (R.F32, R.F32), "bf16": (R.F32, R.BF16)}.items():
            if name == args.precision:
                continue
            extras[name] = run_rhs_leg(R, P, ctx, cfg, idx, W, Ww, xy, f2, w2, args.steps, args.warmup)
            log(f"[bench] {name}: {extras[name]}")
        extras["ensemble64_fp32"] = run_rhs_leg(R, P, ctx, cfg, idx, W, Ww, xy, R.F32, R.F32,
                                                max(args.steps // 10, 5), 2, ensemble=64)
        log(f"[bench] ensemble 64: {extras['ensemble64_fp32']}")
        wcfg = weights_config(1024)
        extras["weights_mixed_1M_fp64"] = weights_leg(R, ctx, wcfg, R.SOLVE_FP64, oracle_ref)
        log(f"[bench] weights fp64: {extras['weights_mixed_1M_fp64']}")
        extras["weights_mixed_1M_fp32_ir"] = weights_leg(R, ctx, wcfg, R.SOLVE_FP32_IR, oracle_ref)
        log(f"[bench] weights fp32+IR: {extras['weights_mixed_1M_fp32_ir']}")
        extras["closure_forward_256x2176"] = closure_leg(R, ctx)
        log(f"[bench] closure: {extras['closure_forward_256x2176']}")
        if not args.no_closure_quality:
            extras["closure_quality_256"] = closure_quality_leg(R, ctx)
            log(f"[bench] closure quality: {extras['closure_quality_256']}")
        extras["device_peaks"] = device_peaks_leg(R, ctx)
        log(f"[bench] device peaks: {extras['device_peaks']}")
        extras["advection_64x64_fp64"] = advection_leg(R, P, ctx)
        log(f"[bench] advection: {extras['advection_64x64_fp64']}")
        if not args.no_fullrun:
            extras["precision_fullrun_900s"] = fullrun_leg(R, P, ctx, cfg, idx, W, Ww, xy)
            log(f"[bench] full runs to 900 s: {extras['precision_fullrun_900s']}")
        # a 4x larger channel (4096 x 512 = 2,097,152 nodes, 2 GB per launch): the
        # bandwidth is not an artefact of the 256 MB Infinity Cache
        big = scale_config(4096, 512)
        _, bidx, bW, bWw, _ = P.ns_weights(ctx, big)
        extras["fp32_4096x512"] = run_rhs_leg(R, P, ctx, big, bidx, bW, bWw, None, R.F32, R.F32,
                                              max(args.steps // 4, 10), 3)
        del bidx, bW, bWw
        log(f"[bench] fp32 4096x512: {extras['fp32_4096x512']}")
    extras["weights_scale_setup"] = dict(stencils=n_stencils, seconds=setup_s,
                                         stencils_per_s=n_stencils / setup_s,
                                         note="search + FP64 weights incl. host sync, 4+2 operators")

    if cpu_weights is not None:
        extras["cpu_oracle_weights"] = cpu_weights

    for name in ("fp64", "fp32", "bf16", "ensemble64_fp32"):
        if name in extras:
            extras[name]["roofline"] = leg_roofline(name, extras[name], nd.n_active)
    k = main_leg
    line = {
        "metric": METRIC,
        "value": k["node_updates_per_s"],
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": k["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "f32 (bf16 weights)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{cfg['name']}: density current, 524,288 active + 4,096 ghost nodes, "
                               f"r^7 + degree-4 polynomials, n=37, RK4 dt=1/16 s, E=1",
                   "stages_per_step": 4, "precision": args.precision},
        "roofline": leg_roofline(args.precision, k, nd.n_active),
        "cpu_baseline": cpu,
        "accuracy": None if "precision_fullrun_900s" not in extras else {
            "theta_rel_l2_at_900s_vs_fp64": {k: extras["precision_fullrun_900s"][k]["theta_rel_l2_vs_fp64"]
                                             for k in ("fp32", "bf16")},
            "note": "same workload run 14,400 RK4 steps to t = 900 s in FP64, FP32 and with BF16 weights"},
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
