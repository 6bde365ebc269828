"""The hot path for the paper's workloads, chained through the C ABI:
node set -> rbffd_knn/rbffd_weights (A1-A4) -> rbffd_model_create ->
rbffd_rhs / rbffd_step (B1-B4). Inputs come from the ``workloads`` package;
every arithmetic step runs in the library's kernels."""

import numpy as np
import torch

from . import rbffd as R


def to_dev(a, dtype=None, device="cuda"):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device)


def ns_ops(cfg):
    return [(R.DX, 0, 0), (R.DZ, 0, 0), (R.LAP, 0, 0), (R.HYPERLAP, cfg["hv_k"], cfg["hv_m"])]


def advection_ops(cfg):
    return [(R.DX, 0, 0), (R.DZ, 0, 0), (R.HYPERLAP, cfg["hv_k"], cfg["hv_m"])]


def ns_weights(ctx, cfg, xy=None):
    """Stencils and weights of a channel or box workload:
    (xy, idx, W, Wwall, status), Wwall [2][R][n] the boundary rows' first and
    second normal-derivative weights (Dz, Dzz on walls normal to z; Dx, Dxx
    on walls normal to x)."""
    nd = cfg["nodes"]
    if xy is None:
        xy = to_dev(nd.xy, torch.float64)
    idx, W, status, _ = R.rbffd_weights(ctx, xy, ns_ops(cfg), cfg["n"], cfg["m"], cfg["l"],
                                        period_x=nd.period_x, n_centers=nd.n_active)
    # the boundary rows repeat the (deterministic) search for their centres
    R_ = len(nd.bnd_nodes)
    Ww = torch.zeros((2, R_, cfg["n"]), dtype=torch.float64, device="cuda")
    wstatus = torch.zeros(R_, dtype=torch.int32, device="cuda")
    for normal, ops in ((0, [(R.DZ, 0, 0), (R.DZZ, 0, 0)]), (1, [(R.DX, 0, 0), (R.DXX, 0, 0)])):
        sel = np.nonzero(nd.bnd_normal == normal)[0]
        if sel.size:
            centers = to_dev(nd.bnd_nodes[sel], torch.int32)
            _, Wn, st, _ = R.rbffd_weights(ctx, xy, ops, cfg["n"], cfg["m"], cfg["l"], period_x=nd.period_x,
                                           centers=centers)
            rows = to_dev(sel, torch.int64)
            Ww[:, rows] = Wn
            wstatus[rows] = st
    return xy, idx, W, Ww, (status, wstatus)


def ns_model(ctx, cfg, idx, W, Ww, xy=None, field_dtype=R.F64, weight_dtype=R.F64, ensemble=1,
             hv_coeff=None):
    nd = cfg["nodes"]
    if xy is None:
        xy = to_dev(nd.xy, torch.float64)
    n = idx.shape[1]
    Ww = Ww.reshape(2, -1, n)
    return R.Model(ctx, R.PHYS_NS, idx, W, xy, nd.n_active, field_dtype=field_dtype,
                   weight_dtype=weight_dtype, ensemble=ensemble,
                   hv_coeff=cfg["hv_coeff"] if hv_coeff is None else hv_coeff, consts=cfg["consts"],
                   bnd_nodes=to_dev(nd.bnd_nodes, torch.int32), bnd_ghosts=to_dev(nd.bnd_ghosts, torch.int32),
                   bnd_normal=to_dev(nd.bnd_normal, torch.int32),
                   bnd_d1=Ww[0].contiguous(), bnd_d2=Ww[1].contiguous())


def advection_model(ctx, cfg, idx, W, xy=None, field_dtype=R.F64, ensemble=1):
    nd = cfg["nodes"]
    if xy is None:
        xy = to_dev(nd.xy, torch.float64)
    src = cfg.get("mirror_src")
    return R.Model(ctx, R.PHYS_ADVECTION, idx, W, xy, nd.n_active, field_dtype=field_dtype,
                   ensemble=ensemble, hv_coeff=cfg["hv_coeff"], vel_u=to_dev(cfg["U"], torch.float64),
                   vel_v=to_dev(cfg["V"], torch.float64), vel_period=cfg["vel_period"],
                   mirror_src=None if src is None else to_dev(src, torch.int32))


def advection_weights(ctx, cfg, xy=None):
    nd = cfg["nodes"]
    if xy is None:
        xy = to_dev(nd.xy, torch.float64)
    idx, W, status, _ = R.rbffd_weights(ctx, xy, advection_ops(cfg), cfg["n"], cfg["m"], cfg["l"],
                                        period_x=nd.period_x, n_centers=nd.n_active)
    return xy, idx, W, status
