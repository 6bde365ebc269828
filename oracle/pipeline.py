"""Oracle pipelines: node set -> stencils -> weights -> right-hand side model,
for the scalar-transport and Navier-Stokes workloads (Sections 3, 5, 6)."""

import numpy as np

from .stencils import knn
from .weights import DX, DZ, LAP, HYPERLAP, DZZ, all_weights
from .rhs import AdvectionModel, NSModel


def advection_ops(cfg):
    return [(DX, 0, 0), (DZ, 0, 0), (HYPERLAP, cfg["hv_k"], cfg["hv_m"])]


def ns_ops(cfg):
    return [(DX, 0, 0), (DZ, 0, 0), (LAP, 0, 0), (HYPERLAP, cfg["hv_k"], cfg["hv_m"])]


def wall_ops():
    return [(DZ, 0, 0), (DZZ, 0, 0)]


def build_advection(cfg):
    nd = cfg["nodes"]
    centers = np.arange(nd.n_active)
    idx = knn(nd.xy, centers, cfg["n"], nd.period_x)
    W, status = all_weights(nd.xy, idx, centers, cfg["m"], cfg["l"], advection_ops(cfg), nd.period_x)
    model = AdvectionModel(idx, W[0], W[1], W[2], cfg["U"], cfg["V"], cfg["hv_coeff"], cfg["vel_period"])
    return model, idx, W, status


def build_ns(cfg, idx=None, W=None, Wwall=None):
    """NSModel for a channel workload. Stencils and weights may be passed in
    (computed elsewhere by the oracle) to save time."""
    nd = cfg["nodes"]
    centers = np.arange(nd.n_active)
    if idx is None:
        idx = knn(nd.xy, centers, cfg["n"], nd.period_x)
    if W is None:
        W, _ = all_weights(nd.xy, idx, centers, cfg["m"], cfg["l"], ns_ops(cfg), nd.period_x)
    wall = nd.wall_nodes.ravel()
    if Wwall is None:
        Wwall, _ = all_weights(nd.xy, idx[wall], wall, cfg["m"], cfg["l"], wall_ops(), nd.period_x)
    nb = nd.wall_nodes.shape[1]
    n = idx.shape[1]
    model = NSModel(idx=idx, w_dx=W[0], w_dz=W[1], w_lap=W[2], w_hv=W[3], z=nd.xy[:, 1].copy(),
                    n_active=nd.n_active, wall_nodes=nd.wall_nodes, ghost_nodes=nd.ghost_nodes,
                    wall_dz=Wwall[0].reshape(-1, nb, n), wall_dzz=Wwall[1].reshape(-1, nb, n),
                    consts=cfg["consts"], hv_coeff=cfg["hv_coeff"])
    return model, idx, W, Wwall
