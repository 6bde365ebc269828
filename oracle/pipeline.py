"""Oracle pipelines: node set -> stencils -> weights -> right-hand side model,
for the scalar-transport and Navier-Stokes workloads (Sections 3, 5, 6)."""

import numpy as np

from .stencils import knn
from .weights import DX, DZ, LAP, HYPERLAP, DZZ, DXX, all_weights
from .rhs import AdvectionModel, NSModel


def advection_ops(cfg):
    return [(DX, 0, 0), (DZ, 0, 0), (HYPERLAP, cfg["hv_k"], cfg["hv_m"])]


def ns_ops(cfg):
    return [(DX, 0, 0), (DZ, 0, 0), (LAP, 0, 0), (HYPERLAP, cfg["hv_k"], cfg["hv_m"])]


def wall_ops(normal=0):
    """First and second derivative along a wall's normal (0: z, 1: x)."""
    return [(DZ, 0, 0), (DZZ, 0, 0)] if normal == 0 else [(DX, 0, 0), (DXX, 0, 0)]


def boundary_weights(cfg, idx):
    """[2][R][n] first/second normal-derivative weights of every boundary row
    (rows of walls normal to z: Dz, Dzz; normal to x: Dx, Dxx)."""
    nd = cfg["nodes"]
    R, n = len(nd.bnd_nodes), idx.shape[1]
    out = np.zeros((2, R, n))
    for normal in (0, 1):
        sel = np.nonzero(nd.bnd_normal == normal)[0]
        if sel.size:
            nodes = nd.bnd_nodes[sel]
            W, _ = all_weights(nd.xy, idx[nodes], nodes, cfg["m"], cfg["l"], wall_ops(normal), nd.period_x)
            out[:, sel] = W
    return out


def build_advection(cfg):
    nd = cfg["nodes"]
    centers = np.arange(nd.n_active)
    idx = knn(nd.xy, centers, cfg["n"], nd.period_x)
    W, status = all_weights(nd.xy, idx, centers, cfg["m"], cfg["l"], advection_ops(cfg), nd.period_x)
    model = AdvectionModel(idx, W[0], W[1], W[2], cfg["U"], cfg["V"], cfg["hv_coeff"], cfg["vel_period"],
                           cfg.get("mirror_src"))
    return model, idx, W, status


def build_ns(cfg, idx=None, W=None, Wwall=None):
    """NSModel for a channel or box workload. Stencils and weights may be
    passed in (computed elsewhere by the oracle) to save time; ``Wwall`` is
    [2][R][n], the boundary rows' first/second normal-derivative weights."""
    nd = cfg["nodes"]
    centers = np.arange(nd.n_active)
    if idx is None:
        idx = knn(nd.xy, centers, cfg["n"], nd.period_x)
    if W is None:
        W, _ = all_weights(nd.xy, idx, centers, cfg["m"], cfg["l"], ns_ops(cfg), nd.period_x)
    if Wwall is None:
        Wwall = boundary_weights(cfg, idx)
    model = NSModel(idx=idx, w_dx=W[0], w_dz=W[1], w_lap=W[2], w_hv=W[3], z=nd.xy[:, 1].copy(),
                    n_active=nd.n_active, bnd_nodes=nd.bnd_nodes, bnd_ghosts=nd.bnd_ghosts,
                    bnd_normal=nd.bnd_normal, bnd_d1=Wwall[0], bnd_d2=Wwall[1],
                    consts=cfg["consts"], hv_coeff=cfg["hv_coeff"])
    return model, idx, W, Wwall
