"""Method-of-lines time stepping.

* ``rk4_step``: the classical 4th-order Runge-Kutta scheme used for every test
  in the paper (Section 6, Section 6.3).
* ``wsrk3_step``: the 3-stage scheme y1 = y + dt/3 f(y), y2 = y + dt/2 f(y1),
  y_next = y + dt f(y2) (stage times t, t + dt/3, t + dt/2); third order for
  linear problems. Offered as the tableau the 3-stage workloads name.
"""

import numpy as np


def rk4_step(f, t, y, dt):
    k1 = f(t, y)
    k2 = f(t + 0.5 * dt, y + 0.5 * dt * k1)
    k3 = f(t + 0.5 * dt, y + 0.5 * dt * k2)
    k4 = f(t + dt, y + dt * k3)
    return y + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def wsrk3_step(f, t, y, dt):
    y1 = y + (dt / 3.0) * f(t, y)
    y2 = y + (dt / 2.0) * f(t + dt / 3.0, y1)
    return y + dt * f(t + dt / 2.0, y2)


def integrate(f, y0, t0, dt, n_steps, tableau="rk4", callback=None):
    step = {"rk4": rk4_step, "wsrk3": wsrk3_step}[tableau]
    y = np.array(y0, dtype=np.float64, copy=True)
    t = t0
    for s in range(n_steps):
        y = step(f, t, y, dt)
        t = t0 + (s + 1) * dt
        if callback is not None:
            callback(s + 1, t, y)
    return y, t
