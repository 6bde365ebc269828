"""Stencil selection: the n nodes nearest to each centre.

The paper uses n-node stencils of nearest nodes (Section 6: n = 37, chosen
because 37 is a complete symmetric set on both Cartesian and hexagonal
lattices, Appendix A). Equal distances are common on lattices, so the order is
fixed by the key (d^2, j): squared distance first, node index second, with
d^2 = dx*dx + dz*dz evaluated in IEEE FP64 as two rounded products and one
rounded sum (no fused multiply-add). For an x-periodic domain dx is the
minimum image: it is shifted by one period when |dx| exceeds half a period.

Parity: pinned by the complete 13- and 37-node shells of Appendix A and by
a pure-Python scalar search on small inputs (tests/test_oracle_stencils.py).
"""

import numpy as np


def min_image(dx: np.ndarray, period: float) -> np.ndarray:
    """x-offset reduced to the nearest periodic image (identity if period==0)."""
    if period <= 0.0:
        return dx
    half = 0.5 * period
    return np.where(dx > half, dx - period, np.where(dx < -half, dx + period, dx))


def knn(xy: np.ndarray, centers, n: int, period_x: float = 0.0) -> np.ndarray:
    """Return int32 [len(centers)][n]: for each centre c, the nodes j of ``xy``
    with the n smallest keys (d^2(c, j), j), in increasing key order."""
    xy = np.asarray(xy, dtype=np.float64)
    centers = np.asarray(centers, dtype=np.int64)
    N = xy.shape[0]
    if n > N:
        raise ValueError("stencil larger than the node set")
    out = np.empty((centers.size, n), dtype=np.int32)
    j_all = np.arange(N)
    for a, c in enumerate(centers):
        dx = min_image(xy[:, 0] - xy[c, 0], period_x)
        dz = xy[:, 1] - xy[c, 1]
        d2 = dx * dx + dz * dz
        # every node whose d^2 does not exceed the n-th smallest value, ties
        # included, then the exact (d^2, j) order on that small set
        thresh = np.partition(d2, n - 1)[n - 1]
        cand = j_all[d2 <= thresh]
        order = np.lexsort((cand, d2[cand]))
        out[a] = cand[order[:n]]
    return out
