"""Learned coarse closure, driven entirely through the C ABI: fine ensemble
runs of the same method, restricted to the coarse nodes, give one-step
correction targets; the network is trained by the library's BF16 matrix-core
kernels; coarse runs with and without the correction are compared with the
fine runs on held-out members."""

import time

import numpy as np
import torch

from . import rbffd as R
from . import pipeline as P


def ensemble_state(cfg, amplitudes, dtype=torch.float32):
    """Initial density-current states [N][E][4], member e with bubble
    amplitude amplitudes[e] (the Eq. Tprime profile scaled)."""
    s0 = cfg["state0"][:, None, :] * (np.asarray(amplitudes) / -15.0)[None, :, None]
    return P.to_dev(s0, dtype).contiguous()


def fine_snapshots(ctx, ccfg, n_coarse_steps):
    """Run the fine ensemble and return its state restricted to the coarse
    active nodes at every coarse step: [n+1][n_active_c][E][4] FP32, plus the
    fine run's wall time."""
    fine = ccfg["fine"]
    E = len(ccfg["amplitudes"])
    xy, idx, W, Ww, _ = P.ns_weights(ctx, fine)
    model = P.ns_model(ctx, fine, idx, W, Ww, xy=xy, field_dtype=R.F32, weight_dtype=R.F32, ensemble=E)
    state = ensemble_state(fine, ccfg["amplitudes"])
    R.rbffd_model_tune(ctx, model, state)  # launch shape only: the same bits in every shape
    fmap = torch.from_numpy(ccfg["fine_of_coarse"]).cuda()
    out = torch.empty((n_coarse_steps + 1, len(ccfg["fine_of_coarse"]), E, 4), dtype=torch.float32, device="cuda")
    out[0] = state[fmap]
    t = 0.0
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for n in range(n_coarse_steps):
        t = R.rbffd_step(ctx, model, state, t, fine["dt"], ccfg["ratio"], R.RK4)
        out[n + 1] = state[fmap]
    torch.cuda.synchronize()
    return out, time.perf_counter() - w0


def coarse_model(ctx, ccfg, E, xy_idx_w=None):
    coarse = ccfg["coarse"]
    if xy_idx_w is None:
        xy_idx_w = P.ns_weights(ctx, coarse)[:4]
    xy, idx, W, Ww = xy_idx_w
    return P.ns_model(ctx, coarse, idx, W, Ww, xy=xy, field_dtype=R.F32, weight_dtype=R.F32, ensemble=E), xy_idx_w


def to_full(model, active):
    """A coarse state [N][E][4] with the given active rows (ghosts zero)."""
    s = torch.zeros(model.state_shape(), dtype=torch.float32, device="cuda")
    s[:active.shape[0]] = active
    return s


def correction_targets(ctx, cmodel, snaps, dt):
    """delta_n = (R u_f(t_{n+1}) - Phi_c(R u_f(t_n))) / dt for n = 0..len-2."""
    tg = torch.empty_like(snaps[:-1])
    for n in range(snaps.shape[0] - 1):
        s = to_full(cmodel, snaps[n])
        R.rbffd_step(ctx, cmodel, s, 0.0, dt, 1, R.RK4)
        tg[n] = (snaps[n + 1] - s[:snaps.shape[1]]) / dt
    return tg


def train(ctx, closure, cmodel, snaps, targets, out_scale, epochs, lr, seed=0, log=None):
    """Adam over the snapshots (one batch = one snapshot, all members)."""
    rng = np.random.default_rng(seed)
    osc = torch.tensor(out_scale, dtype=torch.float32, device="cuda")
    n = targets.shape[0]
    losses = []
    for ep in range(epochs):
        order = rng.permutation(n)
        tot = 0.0
        rate = lr * (0.3 if ep >= int(0.7 * epochs) else 1.0)
        for k in order:
            s = to_full(cmodel, snaps[k])
            R.rbffd_ghost(ctx, cmodel, s)
            tot += closure.train_step(s, (targets[k] / osc).contiguous(), rate)
        losses.append(tot / n)
        if log:
            log(f"[closure] epoch {ep} loss {losses[-1]:.4f}")
    return losses


def rollout_errors(ctx, cmodel, closure, snaps, dt, checkpoints):
    """theta' relative l2 error against the fine run at the checkpoint steps,
    plain coarse run and corrected run (same members as cmodel's)."""
    res = {}
    plain = to_full(cmodel, snaps[0])
    corr = plain.clone()
    t_p = t_c = 0.0
    last = 0
    fallbacks = 0
    for c in checkpoints:
        t_p = R.rbffd_step(ctx, cmodel, plain, t_p, dt, c - last, R.RK4)
        t_c, fb = closure.step(corr, t_c, dt, c - last, R.RK4)
        fallbacks += fb
        last = c
        ref = snaps[c][..., 2]
        na = ref.shape[0]
        ep = torch.linalg.norm(plain[:na, :, 2] - ref) / torch.linalg.norm(ref)
        ec = torch.linalg.norm(corr[:na, :, 2] - ref) / torch.linalg.norm(ref)
        res[int(c)] = (float(ep), float(ec))
    return res, fallbacks


def quality_run(ctx, ccfg, n_steps=150, checkpoints=(30, 60, 120, 150), epochs=30, lr=1e-3, seed=0, log=None):
    """The whole learned part on one closure workload: the fine ensemble's
    snapshots, one-step correction targets, a relu network trained on the
    first n_train members by the library's kernels, then plain and corrected
    coarse runs of the held-out members against their fine runs. Returns the
    theta' relative l2 errors {checkpoint: (plain, corrected)}, the number of
    fallbacks, and timings."""
    say = log or (lambda *a: None)
    snaps, fine_s = fine_snapshots(ctx, ccfg, n_steps)
    E, ntr = len(ccfg["amplitudes"]), ccfg["n_train"]
    say(f"[closure] fine ensemble {E} x {ccfg['fine']['nodes'].n_active} nodes, {n_steps} s: {fine_s:.1f} s")
    cm_all, xyiw = coarse_model(ctx, ccfg, E)
    dt = ccfg["coarse"]["dt"]
    tg = correction_targets(ctx, cm_all, snaps, dt)
    in_scale = [float(snaps[..., c].std()) + 1e-12 for c in range(4)]
    out_scale = [float(tg[:, :, :ntr, c].std()) + 1e-12 for c in range(4)]
    cm_tr, _ = coarse_model(ctx, ccfg, ntr, xyiw)
    nodef = torch.from_numpy(ccfg["node_feature"]).cuda()
    from workloads.fields import closure_init_params
    cl = R.Closure(ctx, cm_tr, torch.from_numpy(closure_init_params(seed)).cuda(), nodef, in_scale, out_scale,
                   activation=R.ACT_RELU)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = train(ctx, cl, cm_tr, snaps[:, :, :ntr].contiguous(), tg[:, :, :ntr].contiguous(), out_scale,
                   epochs=epochs, lr=lr, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    cm_te, _ = coarse_model(ctx, ccfg, E - ntr, xyiw)
    cl_te = R.Closure(ctx, cm_te, cl.params(), nodef, in_scale, out_scale, activation=R.ACT_RELU)
    res, fb = rollout_errors(ctx, cm_te, cl_te, snaps[:, :, ntr:].contiguous(), dt, list(checkpoints))
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    corr = to_full(cm_te, snaps[0, :, ntr:].contiguous())
    cl_te.step(corr, 0.0, dt, n_steps, R.RK4)
    torch.cuda.synchronize()
    corrected_s = time.perf_counter() - w0
    return dict(errors=res, fallbacks=fb, members=E, train_members=ntr, held_out=E - ntr, fine_run_s=fine_s,
                train_s=train_s, corrected_run_s=corrected_s, loss_first=losses[0], loss_last=losses[-1],
                in_scale=in_scale, out_scale=out_scale)
