"""Right-hand sides: sparse differentiation-matrix products, the ghost-node
closure and the PDE right-hand sides.

* ``apply_dm``: the differentiation matrix stores only its nonzeros (Section
  3): row i holds the weights of the stencil of node i, so (D f)_i =
  sum_k w[i][k] f[idx[i][k]].
* ``advection_rhs``: flux-form transport psi_t = -(u psi)_x - (v psi)_y
  (Section 6.1) plus hyperviscosity hv_coeff * Lap^k psi (Section 5.3), with
  velocity (U, V)(x) * cos(pi t / vel_period).
* ``ghost_closure``: Section 5.2. Each boundary row (a boundary node, its
  ghost, and the normal of its wall) carries one equation per field; the
  rows of a differentiation matrix split as W_I u_I + W_B u_B + W_G u_G = bc,
  so u_G = W_G^-1 (bc - W_I u_I - W_B u_B), solved here with a sparse LU of
  W_G (all rows together: near a corner of a box the rows of two walls share
  ghosts). Boundary conditions, with n the wall normal:
  walls normal to z (Section 6.4, Eq. BCbubble): du/dz = dtheta'/dz = 0,
  dpi'/dz = g theta' / (c_p theta_bar (theta_bar + theta')), w = 0 and
  d2w/dz2 = 0; walls normal to x (Section 6.5): u = 0, d2u/dx2 = 0,
  dw/dx = dtheta'/dx = dpi'/dx = 0. Order: w_B (resp. u_B) is set to 0
  first; the four ghost solves are then independent.
* ``ns_rhs``: Eqs. uEq, wEq, thetaEq, piEq with mu * Lap on u, w, theta' and
  hv_coeff * Lap^k on all four fields; dw/dt = 0 on walls normal to z and
  du/dt = 0 on walls normal to x (those values stay 0). A uniform
  background wind u_bar (consts["u_bar"], the translating density current of
  Section 6.4) is added to u in the advective terms.
"""

from dataclasses import dataclass
import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg


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
    CSR form, for long runs. With ``mirror_src`` (Section 6.1 mirror
    boundary) the state also holds ghost nodes n_active.. whose values are
    copies of the active nodes ``mirror_src``; they are refreshed before every
    evaluation and their tendency is 0."""

    def __init__(self, idx, w_dx, w_dy, w_hv, U, V, hv_coeff, vel_period, mirror_src=None):
        self.na = idx.shape[0]
        n = U.shape[0]
        self.Dx, self.Dy, self.Dhv = (dm_matrix(idx, w, n) for w in (w_dx, w_dy, w_hv))
        self.U, self.V, self.hv_coeff, self.vel_period = U, V, hv_coeff, vel_period
        self.mirror_src = mirror_src

    def mirror(self, psi):
        """psi with the ghost values set from their mirror sources."""
        if self.mirror_src is None:
            return psi
        psi = np.array(psi, dtype=np.float64, copy=True)
        psi[self.na:] = psi[self.mirror_src]
        return psi

    def __call__(self, t, psi):
        psi = self.mirror(psi)
        a = np.cos(np.pi * t / self.vel_period)
        out = np.zeros_like(psi)
        out[:self.na] = -(self.Dx @ (self.U * a * psi) + self.Dy @ (self.V * a * psi)) \
            + self.hv_coeff * (self.Dhv @ psi)
        return out


def ghost_matrices(idx, rows_w, bnd_nodes, bnd_ghosts):
    """The ghost block W_G [R][R] (sparse) of one operator per boundary row:
    row r holds the weights ``rows_w[r]`` of the stencil of node
    ``bnd_nodes[r]`` at the ghost columns, column c being ghost
    ``bnd_ghosts[c]``. ``idx`` holds the stencils of at least those nodes
    (``idx[bnd_nodes[r]]``)."""
    col = {int(g): c for c, g in enumerate(bnd_ghosts)}
    R = len(bnd_nodes)
    r_i, c_i, v = [], [], []
    for r, node in enumerate(bnd_nodes):
        for k, j in enumerate(idx[node]):
            c = col.get(int(j))
            if c is not None:
                r_i.append(r)
                c_i.append(c)
                v.append(rows_w[r][k])
    return scipy.sparse.csc_matrix((v, (r_i, c_i)), shape=(R, R))


@dataclass
class WallRows:
    """What the Section 5.2 ghost solve of a node set needs: its boundary
    rows, their stencils and normal-derivative weights, and which nodes are
    ghosts or wall nodes. The stencils of other nodes are not needed."""
    idx: np.ndarray            # [n_active][n] stencils; only the rows of bnd_nodes are read
    n_active: int
    n_total: int
    bnd_nodes: np.ndarray      # [R] boundary node of each boundary row
    bnd_ghosts: np.ndarray     # [R] its ghost
    bnd_normal: np.ndarray     # [R] 0: wall normal to z, 1: wall normal to x
    bnd_d1: np.ndarray         # [R][n] first normal-derivative weights (Dz or Dx)
    bnd_d2: np.ndarray         # [R][n] second normal-derivative weights (Dzz or Dxx)
    consts: dict               # c_p, theta_bar, g

    def __post_init__(self):
        zn = (self.bnd_normal == 0)[:, None]
        self.w_u = np.where(zn, self.bnd_d1, self.bnd_d2)      # du/dz, or d2u/dx2
        self.w_w = np.where(zn, self.bnd_d2, self.bnd_d1)      # d2w/dz2, or dw/dx
        mats = [ghost_matrices(self.idx, W, self.bnd_nodes, self.bnd_ghosts)
                for W in (self.w_u, self.w_w, self.bnd_d1)]
        self.lu = [scipy.sparse.linalg.splu(m) for m in mats] if len(self.bnd_nodes) else []
        ghost = np.zeros(self.n_total, bool)
        ghost[self.bnd_ghosts] = True
        self.is_ghost = ghost
        self.zwall = np.zeros(self.n_active, bool)
        self.zwall[self.bnd_nodes[self.bnd_normal == 0]] = True
        self.xwall = np.zeros(self.n_active, bool)
        self.xwall[self.bnd_nodes[self.bnd_normal == 1]] = True


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
    bnd_nodes: np.ndarray      # [R] boundary node of each boundary row
    bnd_ghosts: np.ndarray     # [R] its ghost
    bnd_normal: np.ndarray     # [R] 0: wall normal to z, 1: wall normal to x
    bnd_d1: np.ndarray         # [R][n] first normal-derivative weights (Dz or Dx)
    bnd_d2: np.ndarray         # [R][n] second normal-derivative weights (Dzz or Dxx)
    consts: dict               # c_p, c_v, R_d, g, theta_bar, mu (u_bar)
    hv_coeff: float

    def __post_init__(self):
        self.walls = WallRows(self.idx, self.n_active, self.z.shape[0], self.bnd_nodes, self.bnd_ghosts,
                              self.bnd_normal, self.bnd_d1, self.bnd_d2, self.consts)
        self.zwall, self.xwall = self.walls.zwall, self.walls.xwall
        # the same differentiation matrices as sparse products, for long runs
        n_tot = self.z.shape[0]
        self.D = [dm_matrix(self.idx, W, n_tot) for W in (self.w_dx, self.w_dz, self.w_lap, self.w_hv)]


def ghost_closure(model, state: np.ndarray) -> np.ndarray:
    """Return a copy of ``state`` [n_total][4] (u, w, theta', pi') with w = 0
    on walls normal to z, u = 0 on walls normal to x, and the ghost rows set
    from the Section 5.2 solve. ``model`` is an NSModel or a WallRows."""
    wr = model.walls if isinstance(model, NSModel) else model
    s = np.array(state, dtype=np.float64, copy=True)
    if not len(wr.bnd_nodes):
        return s
    c = wr.consts
    s[np.nonzero(wr.zwall)[0], 1] = 0.0
    s[np.nonzero(wr.xwall)[0], 0] = 0.0
    nodes = wr.bnd_nodes
    rows = wr.idx[nodes]                                     # [R][n]
    keep = ~wr.is_ghost[rows]                                # non-ghost entries
    th_b = s[nodes, 2]
    bc_pi = np.where(wr.bnd_normal == 0,
                     c["g"] * th_b / (c["c_p"] * c["theta_bar"] * (c["theta_bar"] + th_b)), 0.0)
    for f, W, lu, bc in ((0, wr.w_u, wr.lu[0], 0.0), (1, wr.w_w, wr.lu[1], 0.0),
                         (2, wr.bnd_d1, wr.lu[2], 0.0), (3, wr.bnd_d1, wr.lu[2], bc_pi)):
        r = bc - apply_dm(rows, np.where(keep, W, 0.0), s[:, f])
        s[wr.bnd_ghosts, f] = lu.solve(r)
    return s


def ns_tendency(s, rows, idx, w_dx, w_dz, w_lap, w_hv, z, is_wall, consts, hv_coeff, is_xwall=None,
                derivs=None):
    """Eqs. uEq..piEq at the nodes ``rows`` of a closed state ``s`` [n_total][4]
    (ghost rows filled), given those rows' stencils and weights. ``is_wall``
    marks rows on walls normal to z (dw/dt = 0), ``is_xwall`` rows on walls
    normal to x (du/dt = 0). ``derivs`` may supply the four stencil products
    (Dx s, Dz s, Lap s, Lap^k s, each [rows][4]) computed elsewhere."""
    c = consts
    u, w, th, pi = (s[rows, f] for f in range(4))
    ua = u + c.get("u_bar", 0.0)     # background wind (translating density current)
    if derivs is None:
        D = lambda W: apply_dm(idx, W, s)                # noqa: E731  [rows][4]
        derivs = (D(w_dx), D(w_dz), D(w_lap), D(w_hv))
    dx, dz, lap, hv = derivs
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
    if is_xwall is not None:
        out[is_xwall, 0] = 0.0
    return out


def ns_rhs(model: NSModel, state: np.ndarray):
    """Tendency [n_total][4] of Eqs. uEq..piEq (zero on ghost rows) and the
    closed state (ghost rows filled) it was evaluated on."""
    s = ghost_closure(model, state)
    na = model.n_active
    out = np.zeros_like(s)
    out[:na] = ns_tendency(s, np.arange(na), model.idx, model.w_dx, model.w_dz, model.w_lap,
                           model.w_hv, model.z[:na], model.zwall, model.consts, model.hv_coeff,
                           model.xwall, derivs=[Dm @ s for Dm in model.D])
    return out, s
