"""Diagnostics reported by the paper's tables.

* ``rel_l2``: ||a - b||_2 / ||b||_2 (Fig. convergence_BD caption).
* ``extrema``: min/max of theta' and w (Table tbl:straka).
* ``front_location``: the density-current front is where the -0.5 K contour
  of theta' meets the ground (Table tbl:straka caption). Read here as the
  largest x >= 0 on the bottom wall row where theta' <= -0.5 K, linearly
  interpolated between that node and the next one in x.
"""

import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def extrema(state, n_active):
    th = state[:n_active, 2]
    w = state[:n_active, 1]
    return dict(theta_min=float(th.min()), theta_max=float(th.max()),
                w_min=float(w.min()), w_max=float(w.max()))


def front_location(xy, theta, bottom_nodes, level=-0.5) -> float:
    x = xy[bottom_nodes, 0]
    th = theta[bottom_nodes]
    order = np.argsort(x)
    x, th = x[order], th[order]
    sel = x >= 0.0
    x, th = x[sel], th[sel]
    cold = np.nonzero(th <= level)[0]
    if cold.size == 0:
        return 0.0
    i = cold[-1]
    if i + 1 >= x.size:
        return float(x[i])
    # linear interpolation of the crossing between node i and node i+1
    f = (level - th[i]) / (th[i + 1] - th[i])
    return float(x[i] + f * (x[i + 1] - x[i]))


def translating_fronts(xy, theta, bottom_nodes, center=18000.0, level=-0.5):
    """Table tbl:translating: distances from x = center to the -0.5 K contour
    on the ground on either side (the fronts face each other across the
    centre). Left front: largest x < center with theta' <= level, right
    front: smallest x > center with theta' <= level, each interpolated
    linearly towards the centre."""
    x = xy[bottom_nodes, 0]
    th = theta[bottom_nodes]
    order = np.argsort(x)
    x, th = x[order], th[order]
    cold = th <= level
    left = np.nonzero(cold & (x < center))[0]
    right = np.nonzero(cold & (x > center))[0]
    i, j = left[-1], right[0]
    xl = x[i] + (level - th[i]) / (th[i + 1] - th[i]) * (x[i + 1] - x[i])
    xr = x[j] - (level - th[j]) / (th[j - 1] - th[j]) * (x[j] - x[j - 1])
    return float(center - xl), float(xr - center)


def bubble_height(xy, theta, rows, x0=5000.0, level=0.1):
    """Table tbl:bubble: the height where the ``level`` contour of theta'
    crosses the line x = x0, taken at the top of the bubble. Per node row,
    theta' and z are interpolated linearly in x to x0; the topmost row with
    theta' >= level and the row above it are then interpolated linearly in
    z."""
    zs, ts = [], []
    for r in rows:
        x = xy[r, 0]
        o = np.argsort(x)
        x, z, t = x[o], xy[r, 1][o], theta[r][o]
        k = int(np.searchsorted(x, x0))
        if k == 0 or k == x.size:
            continue
        a = (x0 - x[k - 1]) / (x[k] - x[k - 1])
        zs.append(z[k - 1] + a * (z[k] - z[k - 1]))
        ts.append(t[k - 1] + a * (t[k] - t[k - 1]))
    zs, ts = np.array(zs), np.array(ts)
    top = np.nonzero(ts >= level)[0][-1]
    if top == zs.size - 1:
        return float(zs[top])
    return float(zs[top] + (level - ts[top]) / (ts[top + 1] - ts[top]) * (zs[top + 1] - zs[top]))
