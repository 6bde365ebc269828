"""Initial and synthetic field values for the test cases.

These are problem data, not the method: the cosine bell and swirling velocity
of the scalar-transport test, the cold-bubble temperature perturbation of the
density current (Section 6.4, Eq. Tprime and the theta' = T'/pi-bar relation),
seeded smooth developed states used to compare right-hand sides, and the
ensemble amplitude draw.
"""

import numpy as np

# Section 6.2 constants (and Section 6.4 surface temperature, viscosity).
NS_CONSTANTS = dict(c_p=1004.0, c_v=717.0, R_d=287.0, g=9.81, theta_bar=300.0, mu=75.0)


def cosine_bell(xy: np.ndarray, center=(0.25, 0.5), radius: float = 0.15) -> np.ndarray:
    """(1 + cos(pi r~))/2 for r~ = dist/radius <= 1, else 0 (Section 6.1 bell
    shape; centre and radius are the workload's)."""
    r = np.hypot(xy[:, 0] - center[0], xy[:, 1] - center[1]) / radius
    return np.where(r <= 1.0, 0.5 * (1.0 + np.cos(np.pi * np.minimum(r, 1.0))), 0.0)


def swirl_velocity(xy: np.ndarray):
    """Spatial shape of the reversing deformational flow used by the scalar
    transport workload: U = sin^2(pi x) sin(2 pi y), V = -sin^2(pi y) sin(2 pi x).
    The full velocity is (U, V) * cos(pi t / 5)."""
    x, y = xy[:, 0], xy[:, 1]
    U = np.sin(np.pi * x) ** 2 * np.sin(2.0 * np.pi * y)
    V = -np.sin(np.pi * y) ** 2 * np.sin(2.0 * np.pi * x)
    return U, V


def pi_bar(z: np.ndarray, c=NS_CONSTANTS) -> np.ndarray:
    """Background Exner pressure 1 - g z / (c_p T_s) (Section 6.4)."""
    return 1.0 - c["g"] * z / (c["c_p"] * c["theta_bar"])


def straka_theta(xy: np.ndarray, amplitude: float = -15.0, center=(0.0, 3000.0),
                 radii=(4000.0, 2000.0), c=NS_CONSTANTS) -> np.ndarray:
    """theta' at t=0: T' = amplitude/2 * (1 + cos(pi r)) for r <= 1 (Eq. Tprime
    with amplitude -15 K), divided by pi-bar(z)."""
    x, z = xy[:, 0], xy[:, 1]
    r = np.sqrt(((x - center[0]) / radii[0]) ** 2 + ((z - center[1]) / radii[1]) ** 2)
    T = np.where(r <= 1.0, 0.5 * amplitude * (1.0 + np.cos(np.pi * np.minimum(r, 1.0))), 0.0)
    return T / pi_bar(z, c)


def straka_state(nodes, amplitude: float = -15.0, c=NS_CONSTANTS, dtype=np.float64,
                 center=(0.0, 3000.0)) -> np.ndarray:
    """Initial density-current state [n_total][4] = (u, w, theta', pi'); all
    zero except theta'. Ghost rows are filled by the closure before use."""
    s = np.zeros((nodes.n_total, 4), dtype=np.float64)
    s[:, 2] = straka_theta(nodes.xy, amplitude=amplitude, c=c, center=center)
    s[nodes.n_active:] = 0.0
    return s.astype(dtype)


def bubble_state(nodes, amplitude: float = 2.0, radius: float = 1500.0, center=(5000.0, 3000.0),
                 dtype=np.float64) -> np.ndarray:
    """Rising thermal bubble (Section 6.5): theta' = amplitude * max(0, 1 -
    r / radius), a C0 cone around ``center``; u = w = pi' = 0. Ghost rows are
    filled by the closure before use."""
    s = np.zeros((nodes.n_total, 4), dtype=np.float64)
    r = np.hypot(nodes.xy[:, 0] - center[0], nodes.xy[:, 1] - center[1])
    s[:, 2] = amplitude * np.maximum(0.0, 1.0 - r / radius)
    s[nodes.n_active:] = 0.0
    return s.astype(dtype)


def smooth_ns_state(nodes, seed: int = 2, modes: int = 4, dtype=np.float64) -> np.ndarray:
    """Seeded smooth developed-looking state [n_total][4] on an x-periodic
    channel: u, w ~ 15 m/s, theta' ~ 10 K, pi' ~ 1e-3, built from a few
    Fourier modes in x times cosines (u, theta', pi') or sines (w) in z."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, z = nodes.xy[:, 0], nodes.xy[:, 1]
    L, H = nodes.period_x, nodes.height
    amp = [15.0, 15.0, 10.0, 1e-3]
    s = np.zeros((nodes.n_total, 4))
    for f in range(4):
        for _ in range(modes):
            kx = rng.integers(1, 6)
            kz = rng.integers(0 if f != 1 else 1, 4)
            ph = rng.uniform(0.0, 2.0 * np.pi)
            a = rng.uniform(-1.0, 1.0) * amp[f] / modes
            zf = np.sin(np.pi * kz * z / H) if f == 1 else np.cos(np.pi * kz * z / H)
            s[:, f] += a * np.cos(2.0 * np.pi * kx * x / L + ph) * zf
    s[nodes.n_active:] = 0.0
    return s.astype(dtype)


def ensemble_amplitudes(n_members: int, seed: int = 1, low: float = -17.0, high: float = -13.0):
    """Bubble temperature amplitudes drawn from U[low, high] K (PCG64 seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(low, high, n_members)


def closure_init_params(seed: int = 0, out_rows: int = 4):
    """Seeded initial parameters of the closure network in the C ABI's layout
    (W1 [128][160], b1 [128], W2 [128][128], b2 [128], W3 [16][128], b3 [16]):
    uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights with fan_in 149 for the
    first layer (148 gathered values and one node feature) and 128 after,
    zero biases, zero W3 rows beyond the 4 outputs (PCG64 seed)."""
    hid, kin, nout = 128, 160, 16
    rng = np.random.Generator(np.random.PCG64(seed))
    n = hid * kin + hid + hid * hid + hid + nout * hid + nout
    p = np.zeros(n)
    ow2 = hid * kin + hid
    ow3 = ow2 + hid * hid + hid
    p[:hid * kin] = rng.uniform(-1, 1, hid * kin) / np.sqrt(149.0)
    p[ow2:ow2 + hid * hid] = rng.uniform(-1, 1, hid * hid) / np.sqrt(hid)
    w3 = np.zeros((nout, hid))
    w3[:out_rows] = rng.uniform(-1, 1, (out_rows, hid)) / np.sqrt(hid)
    p[ow3:ow3 + nout * hid] = w3.ravel()
    return p.astype(np.float32)
