"""Write the developed density-current states used by the right-hand-side
parity tests: the oracle alone integrates the hexagonal density current
(Section 6.4 initial state, RK4 at the Section 6.3 time step) from t = 0 to
t = 300 s at 400 m and 200 m, then applies the ghost closure, and the state
[n_total][4] (u, w, theta', pi') is stored in FP64.

    python tests/golden/make_developed_states.py [400 200]
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

T_END = 300.0


def path_for(h):
    return os.path.join(HERE, f"developed_hexagonal_{int(h)}m_{int(T_END)}s.npz")


def make(h):
    import oracle as O
    from oracle.pipeline import build_ns
    from workloads import density_current_config
    cfg = density_current_config("hexagonal", float(h))
    om, _, _, _ = build_ns(cfg)
    n = int(round(T_END / cfg["dt"]))
    f = lambda t, y: O.ns_rhs(om, y)[0]                       # noqa: E731
    y, t = O.integrate(f, cfg["state0"], 0.0, cfg["dt"], n, "rk4")
    y = O.ghost_closure(om, y)
    np.savez_compressed(path_for(h), state=y, t=t, h=float(h), steps=n)
    return y, t


if __name__ == "__main__":
    for h in (sys.argv[1:] or ["400", "200"]):
        y, t = make(float(h))
        print(f"{h} m: t = {t} s, theta' min {y[:, 2].min():.4f} max {y[:, 2].max():.4f}, "
              f"w min {y[:, 1].min():.3f} max {y[:, 1].max():.3f}")
