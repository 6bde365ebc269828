"""Node sets (Section 5.1: Cartesian, hexagonal, quasi-uniform scattered) and
the ghost nodes of Section 5.2, for the paper's test domains.

Ordering convention used everywhere: active nodes (those that carry a stencil
and prognostic values) come first, row by row from the bottom wall upwards,
then the ghost nodes. Every boundary row pairs one boundary node with one
ghost straight outside it and records the wall's normal direction
(``bnd_nodes``, ``bnd_ghosts``, ``bnd_normal``: 0 for a wall normal to z,
1 for a wall normal to x). A corner node of a closed box sits on two walls
and so appears in two boundary rows, with one ghost for each.
"""

from dataclasses import dataclass, field
import numpy as np

KIND_INTERIOR = 0
KIND_WALL = 1          # on a wall normal to z (w = 0 there)
KIND_GHOST = 2
KIND_XWALL = 4         # on a wall normal to x (u = 0 there); corners carry 1 | 4
NORMAL_Z, NORMAL_X = 0, 1


@dataclass
class NodeSet:
    xy: np.ndarray                  # (n_total, 2) float64, [x, z]
    n_active: int                   # nodes 0..n_active-1 have stencils
    period_x: float                 # x period (0.0: not periodic)
    h: float                        # nominal node spacing
    layout: str
    nx: int = 0
    nz: int = 0
    wall_nodes: np.ndarray = field(default_factory=lambda: np.zeros((0, 0), np.int32))
    ghost_nodes: np.ndarray = field(default_factory=lambda: np.zeros((0, 0), np.int32))
    height: float = 0.0
    width: float = 0.0
    bnd_nodes: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    bnd_ghosts: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    bnd_normal: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    rows: list = field(default_factory=list)    # active node indices of each row, bottom up

    @property
    def n_total(self) -> int:
        return int(self.xy.shape[0])

    def kinds(self) -> np.ndarray:
        k = np.zeros(self.n_total, np.int8)
        k[self.n_active:] = KIND_GHOST
        k[self.bnd_nodes[self.bnd_normal == NORMAL_Z]] |= KIND_WALL
        k[self.bnd_nodes[self.bnd_normal == NORMAL_X]] |= KIND_XWALL
        return k


def unit_square_cartesian(n_side: int = 64) -> NodeSet:
    """n_side x n_side Cartesian lattice on [0,1]^2 with x_i = i/(n_side-1);
    node index = j*n_side + i. No ghosts, no periodicity (one-sided stencils
    at the edges)."""
    t = np.arange(n_side, dtype=np.float64) / (n_side - 1)
    X, Y = np.meshgrid(t, t, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1).copy()
    return NodeSet(xy=xy, n_active=xy.shape[0], period_x=0.0, h=1.0 / (n_side - 1),
                   layout="cartesian", nx=n_side, nz=n_side)


def mirrored_square(n_side: int = 64, depth: int = 3) -> NodeSet:
    """The n_side x n_side Cartesian lattice on [0,1]^2 of
    ``unit_square_cartesian`` plus mirror ghosts (Section 6.1): every node
    within ``depth`` spacings of an edge, off that edge, is reflected across
    it (across both edges near a corner, which gives the corner's diagonal
    ghosts too). Ghost k takes the value of active node ``mirror_src[k]``, so
    boundary stencils are mirror-symmetric and need no boundary condition.
    depth = 3 completes the 37-node stencils (shells up to r^2 = 10 h^2)."""
    base = unit_square_cartesian(n_side)
    h = base.h
    lim = depth * h * (1.0 + 1e-9)
    pts, src = [], []
    for i, (x, y) in enumerate(base.xy):
        xs = [x] + ([-x] if 0.0 < x <= lim else []) + ([2.0 - x] if 0.0 < 1.0 - x <= lim else [])
        ys = [y] + ([-y] if 0.0 < y <= lim else []) + ([2.0 - y] if 0.0 < 1.0 - y <= lim else [])
        for a, xv in enumerate(xs):
            for b, yv in enumerate(ys):
                if a or b:
                    pts.append((xv, yv))
                    src.append(i)
    xy = np.concatenate([base.xy, np.array(pts)], axis=0)
    nd = NodeSet(xy=xy, n_active=base.n_active, period_x=0.0, h=h, layout="cartesian", nx=n_side, nz=n_side,
                 height=1.0, width=1.0)
    nd.mirror_src = np.array(src, np.int32)
    return nd


def channel(layout: str, nx: int, nz: int, x_left: float, length: float, height: float,
            seed: int = 0, jitter: float = 0.2) -> NodeSet:
    """x-periodic channel [x_left, x_left+length) x [0, height] with walls at
    z=0 and z=height and one ghost row outside each wall.

    * ``cartesian``: nx columns at spacing hx = length/nx, nz rows at
      dz = height/(nz-1).
    * ``hexagonal``: as Cartesian but odd rows are shifted by hx/2.
    * ``scattered``: hexagonal positions jittered by U[-jitter*hx, jitter*hx]
      in x and z for interior rows, and in x only for wall rows (PCG64 stream
      seeded with ``seed``).

    Ghost node g of a wall is placed straight outside boundary node g (same
    x, one row spacing dz beyond the wall), so every layout gets one ghost per
    boundary node (Section 5.2). On the hexagonal lattice the shifted
    continuation row would not do: a stencil that is symmetric in x weighs
    the two ghosts at -hx/2 and +hx/2 equally, so the alternating ghost mode
    is invisible to every boundary row and W_G is singular.
    """
    if layout not in ("cartesian", "hexagonal", "scattered"):
        raise ValueError(layout)
    hx = length / nx
    dz = height / (nz - 1)
    shifted = layout in ("hexagonal", "scattered")
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = []
    for r in range(nz):
        x = x_left + (np.arange(nx, dtype=np.float64) + (0.5 if (shifted and r % 2) else 0.0)) * hx
        z = np.full(nx, height if r == nz - 1 else r * dz)
        if layout == "scattered":
            x = x + rng.uniform(-jitter * hx, jitter * hx, nx)
            if 0 < r < nz - 1:
                z = z + rng.uniform(-jitter * hx, jitter * hx, nx)
            x = x_left + np.mod(x - x_left, length)
        pts.append(np.stack([x, z], axis=1))
    bottom, top = pts[0], pts[nz - 1]
    pts.append(np.stack([bottom[:, 0], np.full(nx, -dz)], axis=1))
    pts.append(np.stack([top[:, 0], np.full(nx, height + dz)], axis=1))
    xy = np.concatenate(pts, axis=0)
    n_active = nx * nz
    wall = np.stack([np.arange(nx), (nz - 1) * nx + np.arange(nx)]).astype(np.int32)
    ghost = np.stack([n_active + np.arange(nx), n_active + nx + np.arange(nx)]).astype(np.int32)
    return NodeSet(xy=xy, n_active=n_active, period_x=length, h=hx, layout=layout,
                   nx=nx, nz=nz, wall_nodes=wall, ghost_nodes=ghost, height=height, width=length,
                   bnd_nodes=wall.ravel().copy(), bnd_ghosts=ghost.ravel().copy(),
                   bnd_normal=np.zeros(2 * nx, np.int32),
                   rows=[np.arange(r * nx, (r + 1) * nx) for r in range(nz)])


def box(layout: str, h: float, width: float, height: float, seed: int = 0, jitter: float = 0.2) -> NodeSet:
    """Closed box [0, width] x [0, height] with walls on all four sides and one
    ghost straight outside every boundary node of every wall.

    * ``cartesian``: columns x = i h (i = 0 .. width/h), rows h apart.
    * ``hexagonal``: rows about h sqrt(3)/2 apart (count rounded so that the
      top wall is a row); even rows x = i h, odd rows shifted by h/2 and
      closed by a node on each lateral wall (x = 0 and x = width).
    * ``scattered``: hexagonal positions jittered by U[-jitter h, jitter h]
      in x and z, wall nodes along their wall only, corners fixed (PCG64
      stream seeded with ``seed``).

    Ghosts of the bottom and top walls sit one row spacing below/above their
    boundary node; ghosts of the lateral walls one spacing h to the left/right.
    """
    if layout not in ("cartesian", "hexagonal", "scattered"):
        raise ValueError(layout)
    ncol = int(round(width / h)) + 1
    if layout == "cartesian":
        nz = int(round(height / h)) + 1
    else:
        nz = int(round(height / (h * np.sqrt(3.0) / 2.0))) + 1
    dz = height / (nz - 1)
    shifted = layout in ("hexagonal", "scattered")
    rng = np.random.Generator(np.random.PCG64(seed))
    pts, rows, start = [], [], 0
    for r in range(nz):
        if shifted and r % 2:
            x = np.concatenate([[0.0], (np.arange(ncol - 1) + 0.5) * h, [width]])
        else:
            x = np.arange(ncol, dtype=np.float64) * h
            x[-1] = width
        z = np.full(x.size, height if r == nz - 1 else r * dz)
        if layout == "scattered":
            side = (x == 0.0) | (x == width)
            if 0 < r < nz - 1:
                x = np.where(side, x, x + rng.uniform(-jitter * h, jitter * h, x.size))
                z = z + rng.uniform(-jitter * h, jitter * h, x.size)
            else:
                x = np.where(side, x, x + rng.uniform(-jitter * h, jitter * h, x.size))
        pts.append(np.stack([x, z], axis=1))
        rows.append(np.arange(start, start + x.size))
        start += x.size
    n_active = start
    bottom, top = rows[0], rows[-1]
    left = np.array([rw[0] for rw in rows])
    right = np.array([rw[-1] for rw in rows])
    act = np.concatenate(pts, axis=0)
    ghosts = [np.stack([act[bottom, 0], np.full(bottom.size, -dz)], axis=1),
              np.stack([act[top, 0], np.full(top.size, height + dz)], axis=1),
              np.stack([np.full(nz, -h), act[left, 1]], axis=1),
              np.stack([np.full(nz, width + h), act[right, 1]], axis=1)]
    xy = np.concatenate([act] + ghosts, axis=0)
    bnd = np.concatenate([bottom, top, left, right]).astype(np.int32)
    normal = np.concatenate([np.zeros(bottom.size + top.size), np.ones(2 * nz)]).astype(np.int32)
    return NodeSet(xy=xy, n_active=n_active, period_x=0.0, h=h, layout=layout, nx=ncol, nz=nz,
                   height=height, width=width, bnd_nodes=bnd,
                   bnd_ghosts=(n_active + np.arange(bnd.size)).astype(np.int32), bnd_normal=normal, rows=rows)


def straka_nodes(layout: str, h: float, seed: int = 0) -> NodeSet:
    """Density-current domain [-25.6, 25.6] x [0, 6.4] km (Section 6.4) at node
    spacing h metres. Cartesian rows are h apart; hexagonal and scattered rows
    are about h*sqrt(3)/2 apart, the row count rounded so the walls are rows."""
    length, height = 51200.0, 6400.0
    nx = int(round(length / h))
    if layout == "cartesian":
        nz = int(round(height / h)) + 1
    else:
        nz = int(round(height / (h * np.sqrt(3.0) / 2.0))) + 1
    return channel(layout, nx, nz, -25600.0, length, height, seed=seed)


def jittered_square(n_side: int = 1024, seed: int = 0, jitter: float = 0.2) -> NodeSet:
    """n_side^2 quasi-uniform scattered nodes in [0,1]^2: a Cartesian lattice
    with spacing h = 1/(n_side-1), interior nodes jittered by U[-jitter*h,
    jitter*h]^2, edge nodes jittered along their edge only, corners fixed."""
    h = 1.0 / (n_side - 1)
    base = unit_square_cartesian(n_side)
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.uniform(-jitter * h, jitter * h, size=base.xy.shape)
    x, y = base.xy[:, 0], base.xy[:, 1]
    on_x_edge = (x == 0.0) | (x == 1.0)
    on_y_edge = (y == 0.0) | (y == 1.0)
    d[on_x_edge, 0] = 0.0
    d[on_y_edge, 1] = 0.0
    xy = base.xy + d
    return NodeSet(xy=xy, n_active=xy.shape[0], period_x=0.0, h=h, layout="scattered",
                   nx=n_side, nz=n_side)
