"""The five workload shapes (scalar transport, density current at 100 m, batched
weights on 1M scattered nodes, density current at 25 m with ensembles, coarse
400 m density current) as plain dictionaries of method parameters and inputs.

Method parameters follow the paper's problem statement: PHS order m (odd),
polynomial degree l, stencil size n, operators, hyperviscosity power k and
coefficient, viscosity mu, time step (Section 6.3 time-step table) and the
Runge-Kutta tableau.
"""

import numpy as np

from .nodes import unit_square_cartesian, straka_nodes, channel, jittered_square
from .fields import NS_CONSTANTS, cosine_bell, swirl_velocity, straka_state, smooth_ns_state

# Nominal magnitude of the grid-scale symbol of a unit-spacing Laplacian cubed
# ((2 pi^2)^3 rounded); used only to turn a damping rate into a coefficient.
SIGMA_REF = 8000.0
# Hyperviscosity strength for the Navier-Stokes workloads: the grid-scale
# mode is damped at rate NS_HV_C / dt. The paper's scaling rule is garbled;
# 2^-2 is the smallest power of two that keeps the 400 m density current
# stable to 900 s with RK4 at the paper's time step.
NS_HV_C = 0.25

# Section 6.3 time-step table: node spacing (m) -> dt (s); dt halves with h,
# which gives the 12.5 m reference runs (Section 6.5) 1/32 s.
DT_TABLE = {800.0: 2.0, 400.0: 1.0, 200.0: 0.5, 100.0: 0.25, 50.0: 0.125, 25.0: 0.0625, 12.5: 0.03125}


def advection_config(n_side: int = 64, mirror: bool = False):
    """Scalar transport: Cartesian n_side^2 on [0,1]^2, r^5 + degree-4
    polynomials (15 terms), 37-node stencils, Dx, Dy and Laplacian-cubed
    hyperviscosity (HV PHS order 7), RK4 with dt = 2.5e-3 to T = 5. With
    ``mirror`` the edges get mirror ghosts (Section 6.1) instead of one-sided
    stencils; the velocity is the same analytic field at every node."""
    from .nodes import mirrored_square
    nodes = mirrored_square(n_side) if mirror else unit_square_cartesian(n_side)
    U, V = swirl_velocity(nodes.xy)
    h = nodes.h
    return dict(
        name=f"advection-cartesian-{n_side}x{n_side}" + ("-mirror" if mirror else ""),
        nodes=nodes, m=5, l=4, n=37, hv_k=3, hv_m=7,
        hv_coeff=2.0 ** -6 * h ** 6,
        U=U, V=V, vel_period=5.0,
        psi0=cosine_bell(nodes.xy),
        mirror_src=getattr(nodes, "mirror_src", None),
        dt=2.5e-3, t_end=5.0, tableau="rk4",
    )


def density_current_config(layout: str = "hexagonal", h: float = 100.0, seed: int = 0,
                           tableau: str = "rk4"):
    """Straka density current (Section 6.4): r^7 + degree-4 polynomials, n=37,
    operators Dx, Dz, Laplacian and Laplacian-cubed (+ Dz, Dzz at walls),
    mu = 75 m^2/s, dt from the Section 6.3 table, run to t = 900 s."""
    nodes = straka_nodes(layout, h, seed=seed)
    dt = DT_TABLE[float(h)]
    return _ns_config(nodes, f"density-current-{layout}-{int(h)}m", dt, tableau)


def translating_config(layout: str = "hexagonal", h: float = 100.0, seed: int = 0, tableau: str = "rk4"):
    """Translating density current (Section 6.4): as the density current but
    on [0, 36] x [0, 6.4] km with a background wind u_bar = 20 m/s and the
    bubble centred at x = 18 km, so that at 900 s the two fronts face each
    other across x = 18 km."""
    length, height = 36000.0, 6400.0
    nx = int(round(length / h))
    nz = int(round(height / h)) + 1 if layout == "cartesian" else int(round(height / (h * np.sqrt(3.0) / 2.0))) + 1
    nodes = channel(layout, nx, nz, 0.0, length, height, seed=seed)
    cfg = _ns_config(nodes, f"translating-density-current-{layout}-{int(h)}m", DT_TABLE[float(h)], tableau)
    cfg["consts"]["u_bar"] = 20.0
    cfg["state0"] = straka_state(nodes, c=cfg["consts"], center=(18000.0, 3000.0))
    return cfg


def bubble_config(layout: str = "cartesian", h: float = 200.0, seed: int = 0, mu: float = 10.0,
                  tableau: str = "rk4"):
    """Rising thermal bubble (Section 6.5): the closed box [0, 10] x [0, 10]
    km with walls on all four sides, mu = 10 m^2/s, a warm 2 K cone of radius
    1.5 km at (5, 3) km, run to t = 1100 s with the time step of Section
    6.3's table."""
    from .nodes import box
    from .fields import bubble_state
    nodes = box(layout, h, 10000.0, 10000.0, seed=seed)
    cfg = _ns_config(nodes, f"rising-bubble-{layout}-{int(h)}m", DT_TABLE[float(h)], tableau)
    cfg["consts"]["mu"] = mu
    cfg["t_end"] = 1100.0
    cfg["state0"] = bubble_state(nodes)
    return cfg


def scale_config(nx: int = 2048, nz: int = 256, tableau: str = "rk4"):
    """Density current on a 2048 x 256 hexagonal-row channel at 25 m column
    spacing (rows at 6400/255 m), 524,288 active nodes plus 2 x 2048 ghosts.
    Other sizes keep the domain; dt follows the column spacing (1/16 s at
    25 m, as in Section 6.3's table)."""
    nodes = channel("hexagonal", nx, nz, -25600.0, 51200.0, 6400.0)
    dt = 0.0625 * (51200.0 / nx) / 25.0
    return _ns_config(nodes, f"density-current-hexagonal-{nx}x{nz}", dt, tableau)


def _ns_config(nodes, name, dt, tableau):
    c = dict(NS_CONSTANTS)
    h = nodes.h
    return dict(
        name=name, nodes=nodes, m=7, l=4, n=37, hv_k=3, hv_m=7,
        hv_coeff=NS_HV_C * h ** 6 / (SIGMA_REF * dt),
        consts=c, dt=dt, t_end=900.0, tableau=tableau,
        state0=straka_state(nodes, c=c),
    )


def weights_config(n_side: int = 1024, seed: int = 0):
    """Batched weights on n_side^2 jittered-Cartesian nodes in [0,1]^2:
    per-node degree l ~ U{3,4,5}, PHS order m = 2l-3, stencil size n = 2M+1
    (interior) or 2M+19 (within 3h of an edge), M = (l+1)(l+2)/2;
    operators Dx, Dy and Laplacian^k with k = (m-1)/2."""
    nodes = jittered_square(n_side, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    l = rng.integers(3, 6, nodes.n_active).astype(np.int32)
    M = (l + 1) * (l + 2) // 2
    x, y = nodes.xy[:, 0], nodes.xy[:, 1]
    edge = np.minimum(np.minimum(x, 1.0 - x), np.minimum(y, 1.0 - y)) < 3.0 * nodes.h
    n = np.where(edge, 2 * M + 19, 2 * M + 1).astype(np.int32)
    m = (2 * l - 3).astype(np.int32)
    return dict(name=f"weights-scattered-{n_side}x{n_side}", nodes=nodes,
                l_per=l, m_per=m, n_per=n, n_max=int(n.max()))


def smooth_state_for(nodes, seed: int = 2, dtype=np.float64):
    return smooth_ns_state(nodes, seed=seed, dtype=dtype)


def closure_config(n_members: int = 64, n_train: int = 48, seed: int = 1, coarse_h: float = 400.0,
                   fine_h: float = 50.0):
    """Learned-closure workload: the density current on nested Cartesian node
    sets -- coarse 400 m (128 x 17 nodes, dt = 1 s) and fine 50 m
    (1024 x 129, dt = 1/8 s), every coarse node also a fine node -- with an
    ensemble whose bubble amplitudes are drawn from U[-17, -13] K. The first
    n_train members train the network, the rest judge it."""
    from .fields import ensemble_amplitudes
    coarse = density_current_config("cartesian", coarse_h)
    fine = density_current_config("cartesian", fine_h)
    cn, fn = coarse["nodes"], fine["nodes"]
    r = int(round(coarse_h / fine_h))
    ci = np.arange(cn.n_active)
    col, row = ci % cn.nx, ci // cn.nx
    fmap = (row * r) * fn.nx + col * r
    assert np.allclose(fn.xy[fmap], cn.xy[:cn.n_active])
    amps = ensemble_amplitudes(n_members, seed=seed)
    return dict(name=f"closure-density-current-cartesian-{int(coarse_h)}m-from-{int(fine_h)}m",
                coarse=coarse, fine=fine, fine_of_coarse=fmap, amplitudes=amps, n_train=n_train,
                node_feature=cn.xy[:cn.n_active, 1] / cn.height, ratio=r)
