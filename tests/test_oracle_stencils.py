"""Pins of the oracle's stencil search (Section 6, Appendix A)."""

import csv
import math
import os
import random

import numpy as np

import oracle as O
from workloads import unit_square_cartesian, channel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _hex_patch(n=21):
    """A true hexagonal lattice (rows sqrt(3)/2 apart, odd rows shifted 1/2)."""
    pts = []
    for j in range(n):
        for i in range(n):
            pts.append((i + 0.5 * (j % 2), j * math.sqrt(3.0) / 2.0))
    return np.array(pts)


def _shells():
    with open(os.path.join(GOLDEN, "shells.csv")) as f:
        rows = [r for r in csv.reader(f) if r and not r[0].startswith("#")]
    return [(r[0], int(r[1]), float(r[2])) for r in rows[1:]]


def test_complete_symmetric_shells():
    """Appendix A: 13 and 37 are complete shells on both lattices, so the
    n-NN stencil of an interior node is exactly the disc of that radius."""
    cart = unit_square_cartesian(21).xy * 20.0       # unit spacing
    hexp = _hex_patch(21)
    for lattice, n, r2 in _shells():
        xy = cart if lattice == "cartesian" else hexp
        c = 10 * 21 + 10
        st = O.knn(xy, [c], n)[0]
        d2 = np.sum((xy[st] - xy[c]) ** 2, axis=1)
        disc = np.nonzero(np.sum((xy - xy[c]) ** 2, axis=1) <= r2 + 1e-9)[0]
        assert sorted(st.tolist()) == sorted(disc.tolist()), (lattice, n)
        assert st[0] == c and np.all(np.diff(d2) >= -1e-12)


def _scalar_knn(xy, c, n, period):
    """Pure-Python scalar search: every node, key (d2, j)."""
    keys = []
    for j in range(len(xy)):
        dx = xy[j][0] - xy[c][0]
        if period > 0:
            if dx > period / 2:
                dx -= period
            elif dx < -period / 2:
                dx += period
        dz = xy[j][1] - xy[c][1]
        a = dx * dx
        b = dz * dz
        keys.append((a + b, j))
    keys.sort()
    return [j for _, j in keys[:n]]


def test_matches_scalar_search_with_ties_and_wrap():
    nd = channel("cartesian", 12, 6, -6.0, 12.0, 5.0)     # unit spacing: many ties
    xy = nd.xy.tolist()
    for c in range(nd.n_active):
        got = O.knn(nd.xy, [c], 13, nd.period_x)[0].tolist()
        assert got == _scalar_knn(xy, c, 13, nd.period_x), c
    rng = random.Random(3)
    pts = np.array([[rng.random(), rng.random()] for _ in range(80)])
    for c in range(0, 80, 7):
        assert O.knn(pts, [c], 21)[0].tolist() == _scalar_knn(pts.tolist(), c, 21, 0.0)


def test_periodic_wrap_equals_shifted_copy():
    """A centre at the left end of an x-periodic channel sees the right end as
    neighbours: same distances as in a copy shifted by half a period."""
    nd = channel("hexagonal", 32, 9, 0.0, 32.0, 8.0)
    c = 4 * 32                                         # left end of row 4
    st = O.knn(nd.xy, [c], 37, nd.period_x)[0]
    shifted = nd.xy.copy()
    shifted[:, 0] = np.mod(shifted[:, 0] + 16.0, 32.0)
    st2 = O.knn(shifted, [c], 37, 0.0)[0]
    assert sorted(st.tolist()) == sorted(st2.tolist())
    assert np.any(nd.xy[st, 0] > 20.0)                 # some come from the right end
