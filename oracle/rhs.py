"""Right-hand sides: sparse differentiation-matrix products, the ghost-node
closure and the PDE right-hand sides.

* ``apply_dm``: the differentiation matrix stores only its nonzeros (Section
  3): row i holds the weights of the stencil of node i, so (D f)_i =
  sum_k w[i][k] f[idx[i][k]].
* ``advection_rhs``: flux-form transport psi_t = -(u psi)_x - (v psi)_y
  (Section 6.1) plus hyperviscosity hv_coeff * Lap^k psi (Section 5.3), with
  velocity (U, V)(x) * cos(pi t / vel_period).
* ``ghost_closure``: Section 5.2. For each wall and boundary condition the
  boundary-node rows of a differentiation matrix split as
  W_I u_I + W_B u_B + W_G u_G = bc, so u_G = W_G^-1 (bc - W_I u_I - W_B u_B),
  solved here with a dense LU of W_G. Section 6.4 boundary conditions:
  du/dz = dtheta'/dz = 0, dpi'/dz = g theta' / (c_p theta_bar (theta_bar +
  theta')), w = 0 and d2w/dz2 = 0. Order: w_B is set to 0 first; the four
  ghost solves are then independent.
* ``ns_rhs``: Eqs. uEq, wEq, thetaEq, piEq with mu * Lap on u, w, theta' and
  hv_coeff * Lap^k on all four fields; dw/dt = 0 on the walls (w_B stays 0).
  A uniform background wind u_bar (consts["u_bar"], the translating density
  current of Section 6.4) is added to u in the advective terms.
"""

from dataclasses import dataclass
import numpy as np
import scipy.linalg
import scipy.sparse


def apply_dm(idx: np.ndarray, w: np.ndarray, f: np.ndarray) -> np.ndarray:
    """sum_k w[i][k] * f[idx[i][k]] for every row i (f may carry trailing axes)."""
    g = f[idx]                                   # (rows, n, ...)
    wb = w.reshape(w.shape + (1,) * (g.ndim - 2))
    return np.sum(wb * g, axis=1)


def dm_matrix(idx: np.ndarray, w: np.ndarray, n_cols: int):
    """The same differentiation matrix as a scipy CSR matrix (duplicates are
    summed, as in the row sum of ``apply_dm``)."""
    rows = np.repeat(np.arange(idx.shape[0]), idx.shape[1])
    return scipy.sparse.csr_matrix((w.ravel(), (rows, idx.ravel())), shape=(idx.shape[0], n_cols))


def advection_rhs(t, psi, idx, w_dx, w_dy, w_hv, U, V, hv_coeff, vel_period):
    """Section 6.1 transport equation in flux form plus hyperviscosity."""
    a = np.cos(np.pi * t / vel_period)
    u = U * a
    v = V * a
    return -(apply_dm(idx, w_dx, u * psi) + apply_dm(idx, w_dy, v * psi)) \
        + hv_coeff * apply_dm(idx, w_hv, psi)


class AdvectionModel:
    """``advection_rhs`` with the three differentiation matrices prebuilt in
    CSR form, for long runs."""

    def __init__(self, idx, w_dx, w_dy, w_hv, U, V, hv_coeff, vel_period):
        n = idx.shape[0]
        self.Dx, self.Dy, self.Dhv = (dm_matrix(idx, w, n) for w in (w_dx, w_dy, w_hv))
        self.U, self.V, self.hv_coeff, self.vel_period = U, V, hv_coeff, vel_period

    def __call__(self, t, psi):
        a = np.cos(np.pi * t / self.vel_period)
        return -(self.Dx @ (self.U * a * psi) + self.Dy @ (self.V * a * psi)) \
            + self.hv_coeff * (self.Dhv @ psi)


def ghost_matrices(idx, w_wall, wall_nodes, ghost_nodes):
    """Split the wall rows of a differentiation matrix (weights ``w_wall``
    [n_walls][n_wall][n] at the nodes ``wall_nodes``) into the ghost block
    W_G [n_walls][n_wall][n_wall] and the rest. Returns W_G."""
    n_walls, nb = wall_nodes.shape
    WG = np.zeros((n_walls, nb, nb))
    for wl in range(n_walls):
        pos = {int(g): p for p, g in enumerate(ghost_nodes[wl])}
        others = set(int(g) for o in range(n_walls) if o != wl for g in ghost_nodes[o])
        for b, node in enumerate(wall_nodes[wl]):
            for k, j in enumerate(idx[node]):
                j = int(j)
                if j in pos:
                    WG[wl, b, pos[j]] += w_wall[wl, b, k]
                elif j in others:
                    raise ValueError("a wall stencil reaches the other wall's ghosts")
    return WG


@dataclass
class NSModel:
    """Everything the Navier-Stokes right-hand side needs (FP64)."""
    idx: np.ndarray            # [n_active][n] stencils
    w_dx: np.ndarray           # [n_active][n]
    w_dz: np.ndarray
    w_lap: np.ndarray
    w_hv: np.ndarray
    z: np.ndarray              # [n_total] node heights
    n_active: int
    wall_nodes: np.ndarray     # [n_walls][n_wall]
    ghost_nodes: np.ndarray    # [n_walls][n_wall]
    wall_dz: np.ndarray        # [n_walls][n_wall][n] Dz weights at wall nodes
    wall_dzz: np.ndarray       # [n_walls][n_wall][n] Dzz weights at wall nodes
    consts: dict               # c_p, c_v, R_d, g, theta_bar, mu
    hv_coeff: float

    def __post_init__(self):
        self.WG_dz = ghost_matrices(self.idx, self.wall_dz, self.wall_nodes, self.ghost_nodes)
        self.WG_dzz = ghost_matrices(self.idx, self.wall_dzz, self.wall_nodes, self.ghost_nodes)
        self.lu_dz = [scipy.linalg.lu_factor(m) for m in self.WG_dz]
        self.lu_dzz = [scipy.linalg.lu_factor(m) for m in self.WG_dzz]
        ghost = np.zeros(self.z.shape[0], bool)
        ghost[self.ghost_nodes.ravel()] = True
        self.is_ghost = ghost


def ghost_closure(model: NSModel, state: np.ndarray) -> np.ndarray:
    """Return a copy of ``state`` [n_total][4] (u, w, theta', pi') with w = 0
    on the walls and the ghost rows set from the Section 5.2 solve."""
    s = np.array(state, dtype=np.float64, copy=True)
    c = model.consts
    s[model.wall_nodes.ravel(), 1] = 0.0
    for wl in range(model.wall_nodes.shape[0]):
        nodes = model.wall_nodes[wl]
        rows = model.idx[nodes]                              # [n_wall][n]
        keep = ~model.is_ghost[rows]                         # non-ghost entries
        wz = np.where(keep, model.wall_dz[wl], 0.0)
        wzz = np.where(keep, model.wall_dzz[wl], 0.0)
        th_b = s[nodes, 2]
        bc = {0: 0.0, 1: 0.0, 2: 0.0,
              3: c["g"] * th_b / (c["c_p"] * c["theta_bar"] * (c["theta_bar"] + th_b))}
        for f in range(4):
            if f == 1:
                r = -apply_dm(rows, wzz, s[:, 1])
                g = scipy.linalg.lu_solve(model.lu_dzz[wl], r)
            else:
                r = bc[f] - apply_dm(rows, wz, s[:, f])
                g = scipy.linalg.lu_solve(model.lu_dz[wl], r)
            s[model.ghost_nodes[wl], f] = g
    return s


def ns_tendency(s, rows, idx, w_dx, w_dz, w_lap, w_hv, z, is_wall, consts, hv_coeff):
    """Eqs. uEq..piEq at the nodes ``rows`` of a closed state ``s`` [n_total][4]
    (ghost rows filled), given those rows' stencils and weights."""
    c = consts
    u, w, th, pi = (s[rows, f] for f in range(4))
    ua = u + c.get("u_bar", 0.0)     # background wind (translating density current)
    D = lambda W: apply_dm(idx, W, s)                    # noqa: E731  [rows][4]
    dx, dz, lap, hv = D(w_dx), D(w_dz), D(w_lap), D(w_hv)
    pibar = 1.0 - c["g"] * z / (c["c_p"] * c["theta_bar"])
    dpibar = -c["g"] / (c["c_p"] * c["theta_bar"])
    out = np.zeros((len(rows), 4))
    cp_th = c["c_p"] * (c["theta_bar"] + th)
    out[:, 0] = -ua * dx[:, 0] - w * dz[:, 0] - cp_th * dx[:, 3] + c["mu"] * lap[:, 0]
    out[:, 1] = -ua * dx[:, 1] - w * dz[:, 1] - cp_th * dz[:, 3] \
        + c["g"] * th / c["theta_bar"] + c["mu"] * lap[:, 1]
    out[:, 2] = -ua * dx[:, 2] - w * dz[:, 2] + c["mu"] * lap[:, 2]
    out[:, 3] = -ua * dx[:, 3] - w * (dpibar + dz[:, 3]) \
        - (c["R_d"] / c["c_v"]) * (pibar + pi) * (dx[:, 0] + dz[:, 1])
    out += hv_coeff * hv
    out[is_wall, 1] = 0.0
    return out


def ns_rhs(model: NSModel, state: np.ndarray):
    """Tendency [n_total][4] of Eqs. uEq..piEq (zero on ghost rows) and the
    closed state (ghost rows filled) it was evaluated on."""
    s = ghost_closure(model, state)
    na = model.n_active
    is_wall = np.zeros(na, bool)
    is_wall[model.wall_nodes.ravel()] = True
    out = np.zeros_like(s)
    out[:na] = ns_tendency(s, np.arange(na), model.idx, model.w_dx, model.w_dz, model.w_lap,
                           model.w_hv, model.z[:na], is_wall, model.consts, model.hv_coeff)
    return out, s
