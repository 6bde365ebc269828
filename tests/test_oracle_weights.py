"""Pins of the oracle's weights (Section 3 Eq. weights, Section 4, Section 5.3
Eq. eqn:laplacian) against things fixed independently of its code."""

import csv
import math
import os

import mpmath
import numpy as np
import pytest
import sympy as sp

import oracle as O
from oracle.weights import poly_exponents
from workloads import unit_square_cartesian, jittered_square, channel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
OPS = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.LAP, 0, 0), (O.DZZ, 0, 0), (O.DXX, 0, 0)]


def test_unisolvent_case_is_central_differences():
    """n = M (6 nodes, degree 2): the polynomial interpolant is unique, so the
    weights are the textbook central differences for any PHS order."""
    xy = np.array([[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1], [1, 1]], float)
    with open(os.path.join(GOLDEN, "central_fd.csv")) as f:
        rows = [r for r in csv.reader(f) if r and not r[0].startswith("#")][1:]
    kinds = {"dx": O.DX, "dz": O.DZ, "lap": O.LAP}
    for m in (3, 5, 7, 9):
        W, st = O.stencil_weights(xy, np.arange(6), 0, m, 2, [(kinds[r[0]], 0, 0) for r in rows])
        assert st == 0
        for w, r in zip(W, rows):
            np.testing.assert_allclose(w, [float(v) for v in r[1:]], atol=1e-13)


def _sym_ops(m, k):
    """Operators applied to ||x - y||^m with sympy (independent route)."""
    x, z, a, b = sp.symbols("x z a b", real=True)
    phi = ((x - a) ** 2 + (z - b) ** 2) ** sp.Rational(m, 2)
    lap = lambda f: sp.diff(f, x, 2) + sp.diff(f, z, 2)        # noqa: E731
    hk = phi
    for _ in range(k):
        hk = lap(hk)
    exprs = {O.DX: sp.diff(phi, x), O.DZ: sp.diff(phi, z), O.LAP: lap(phi),
             O.DZZ: sp.diff(phi, z, 2), O.DXX: sp.diff(phi, x, 2), O.HYPERLAP: hk}
    return {kk: sp.lambdify((a, b), e.subs({x: 0, z: 0}), "mpmath") for kk, e in exprs.items()}


@pytest.mark.parametrize("m,k", [(3, 1), (5, 2), (7, 3), (7, 2), (9, 3)])
def test_operator_rhs_matches_symbolic_derivatives(m, k):
    """Eq. eqn:laplacian applied k times, and the first/second derivatives of
    r^m, checked against sympy's derivatives at sample offsets."""
    f = _sym_ops(m, k)
    rng = np.random.default_rng(5)
    pts = rng.uniform(-1, 1, (12, 2))
    for kind in (O.DX, O.DZ, O.LAP, O.DZZ, O.DXX, O.HYPERLAP):
        got = O.phs_apply(kind, m, k, pts[:, 0], pts[:, 1])
        ref = np.array([float(f[kind](p[0], p[1])) for p in pts])
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)
    # the centre (r = 0) entry is zero for every operator
    for kind in (O.DX, O.DZ, O.LAP, O.DZZ, O.DXX, O.HYPERLAP):
        assert O.phs_apply(kind, m, k, np.zeros(1), np.zeros(1))[0] == 0.0


def test_poly_rows_match_symbolic():
    x, z = sp.symbols("x z")
    for k in (1, 2, 3):
        for (a, b) in poly_exponents(6):
            e = x ** a * z ** b
            h = e
            for _ in range(k):
                h = sp.diff(h, x, 2) + sp.diff(h, z, 2)
            assert O.poly_apply(O.HYPERLAP, k, a, b) == float(h.subs({x: 0, z: 0}))
            assert O.poly_apply(O.DZZ, 0, a, b) == float(sp.diff(e, z, 2).subs({x: 0, z: 0}))
            assert O.poly_apply(O.DXX, 0, a, b) == float(sp.diff(e, x, 2).subs({x: 0, z: 0}))


def _stencils():
    """(xy, stencil, centre, period) samples: interior, edge and corner of a
    jittered square; interior and wall of a periodic hexagonal channel."""
    sq = jittered_square(24, seed=4)
    ch = channel("hexagonal", 40, 9, -20.0, 40.0, 8.0 * math.sqrt(3) / 2)
    out = []
    for c in (12 * 24 + 11, 24 * 2 + 12, 0, 23):
        out.append((sq.xy, c, 0.0))
    for c in (4 * 40 + 3, 0, 8 * 40 + 39):
        out.append((ch.xy, c, ch.period_x))
    return out


@pytest.mark.parametrize("m,l,n", [(3, 3, 21), (5, 4, 31), (7, 4, 37), (7, 5, 43), (3, 5, 61)])
def test_polynomial_reproduction(m, l, n):
    """Section 3: the constraint rows make the weights exact for every
    polynomial of degree <= l, in physical coordinates after rescaling."""
    for xy, c, per in _stencils():
        st = O.knn(xy, [c], n, per)[0]
        ops = OPS + [(O.HYPERLAP, (m - 1) // 2, 0)]
        W, status = O.stencil_weights(xy, st, c, m, l, ops, per)
        assert status == 0
        dx = O.min_image(xy[st, 0] - xy[c, 0], per)
        dz = xy[st, 1] - xy[c, 1]
        for (a, b) in poly_exponents(l):
            vals = dx ** a * dz ** b
            for (kind, k, _), w in zip(ops, W):
                exact = O.poly_apply(kind, k, a, b)
                scale = np.sum(np.abs(w * vals)) + abs(exact)
                assert abs(np.dot(w, vals) - exact) <= 1e-11 * scale, (kind, a, b)


def _mp_exact_weights(xy, st, c, m, l, ops, period):
    """Eq. (weights) formed and solved in 40-digit arithmetic from the FP64
    node coordinates; operator right-hand sides from sympy derivatives."""
    mpmath.mp.dps = 40
    mpf = mpmath.mpf
    d64 = xy[st, 0] - xy[c, 0]
    dx, dz = [], []
    for i, j in enumerate(st):
        shift = 0.0
        if period > 0 and d64[i] > period / 2:
            shift = -period
        elif period > 0 and d64[i] < -period / 2:
            shift = period
        dx.append(mpf(float(xy[j, 0])) - mpf(float(xy[c, 0])) + mpf(shift))
        dz.append(mpf(float(xy[j, 1])) - mpf(float(xy[c, 1])))
    rho = mpmath.sqrt(max(a * a + b * b for a, b in zip(dx, dz)))
    x = [a / rho for a in dx]
    z = [b / rho for b in dz]
    n = len(st)
    exps = poly_exponents(l)
    K = n + len(exps)
    A = mpmath.zeros(K, K)
    for i in range(n):
        for j in range(n):
            A[i, j] = mpmath.sqrt((x[i] - x[j]) ** 2 + (z[i] - z[j]) ** 2) ** m
        for q, (a, b) in enumerate(exps):
            A[i, n + q] = A[n + q, i] = x[i] ** a * z[i] ** b
    X, Z = sp.symbols("X Z")
    out = []
    for kind, k in ops:
        f = _sym_ops(m, k)[kind]
        rhs = mpmath.zeros(K, 1)
        for i in range(n):
            rhs[i] = f(x[i], z[i]) if (x[i] != 0 or z[i] != 0) else mpf(0)
        for q, (a, b) in enumerate(exps):
            e = X ** a * Z ** b
            h = {O.DX: sp.diff(e, X), O.DZ: sp.diff(e, Z), O.LAP: sp.diff(e, X, 2) + sp.diff(e, Z, 2),
                 O.DZZ: sp.diff(e, Z, 2), O.DXX: sp.diff(e, X, 2)}.get(kind)
            if kind == O.HYPERLAP:
                h = e
                for _ in range(k):
                    h = sp.diff(h, X, 2) + sp.diff(h, Z, 2)
            rhs[n + q] = mpf(str(h.subs({X: 0, Z: 0})))
        sol = mpmath.lu_solve(A, rhs)
        scale = rho ** O.op_order(kind, k)
        out.append(np.array([float(sol[i] / scale) for i in range(n)]))
    return out


@pytest.mark.parametrize("m,l,n", [(3, 3, 21), (7, 4, 37), (7, 5, 61)])
def test_exact_solution_40_digits(m, l, n):
    """The oracle reaches the exact solution of Eq. (weights) for the given
    FP64 node positions: compare with the system formed and solved in
    40-digit arithmetic (independent assembly, sympy right-hand sides),
    including one-sided degree-5 stencils whose FP64-rounded system alone
    would move the weights by ~5e-10."""
    for xy, c, per in _stencils()[::2]:
        st = O.knn(xy, [c], n, per)[0]
        ops = [(O.DX, 0), (O.LAP, 0), (O.DXX, 0), (O.HYPERLAP, (m - 1) // 2)]
        W, _ = O.stencil_weights(xy, st, c, m, l, [(kk, k, 0) for kk, k in ops], per)
        ref = _mp_exact_weights(xy, st, c, m, l, ops, per)
        for j in range(len(ops)):
            err = np.linalg.norm(W[j] - ref[j]) / np.linalg.norm(ref[j])
            assert err < 1e-12, (ops[j], err)


def test_symmetry_translation_and_scale():
    """Interior lattice stencils: Dx antisymmetric and Lap^3 symmetric under
    x-mirroring, all interior stencils equal (translation invariance),
    derivative weights sum to zero, and w(sX) = s^-q w(X)."""
    nd = unit_square_cartesian(31)
    ops = [(O.DX, 0, 0), (O.LAP, 0, 0), (O.HYPERLAP, 3, 7)]
    ref = None
    for c in (15 * 31 + 15, 12 * 31 + 14, 17 * 31 + 13):
        st = O.knn(nd.xy, [c], 37)[0]
        W, _ = O.stencil_weights(nd.xy, st, c, 5, 4, ops)
        off = np.round((nd.xy[st] - nd.xy[c]) / nd.h).astype(int)
        key = {tuple(o): i for i, o in enumerate(off)}
        mir = [key[(-o[0], o[1])] for o in off]
        np.testing.assert_allclose(W[0], -W[0][mir], atol=1e-11 * np.abs(W[0]).max())
        np.testing.assert_allclose(W[2], W[2][mir], atol=1e-11 * np.abs(W[2]).max())
        for w in W:
            assert abs(w.sum()) <= 1e-12 * np.abs(w).sum()
        by_off = {tuple(o): W[:, i] for i, o in enumerate(off)}
        if ref is None:
            ref = by_off
        else:
            for o, v in by_off.items():
                np.testing.assert_allclose(v, ref[o], rtol=1e-9, atol=1e-9 * np.abs(W).max())
    c = 15 * 31 + 15
    st = O.knn(nd.xy, [c], 37)[0]
    W1, _ = O.stencil_weights(nd.xy, st, c, 5, 4, ops)
    W2, _ = O.stencil_weights(nd.xy * 8.0, st, c, 5, 4, ops)
    for w1, w2, q in zip(W1, W2, (1, 2, 6)):
        np.testing.assert_allclose(w2, w1 * 8.0 ** (-q), rtol=1e-10, atol=1e-12 * np.abs(w1 * 8.0 ** -q).max())


@pytest.mark.parametrize("m,l", [(3, 3), (3, 4), (7, 3), (7, 4)])
def test_convergence_order_is_degree(m, l):
    """Section 4: d/dx of 1 + sin 4x + cos 3x + sin 2y at the centre of a
    37-node hexagonal stencil converges like h^l for both r^3 and r^7."""
    def lattice(h):
        pts = [((i + 0.5 * (j % 2)) * h, j * h * math.sqrt(3) / 2) for j in range(-6, 7) for i in range(-6, 7)]
        return np.array(pts)
    f = lambda p: 1 + np.sin(4 * p[:, 0]) + np.cos(3 * p[:, 0]) + np.sin(2 * p[:, 1])  # noqa: E731
    x0 = np.array([0.3, -0.2])
    exact = 4 * np.cos(4 * x0[0]) - 3 * np.sin(3 * x0[0])
    hs = [0.1, 0.05, 0.025]
    errs = []
    for h in hs:
        xy = lattice(h) + x0
        c = int(np.argmin(np.sum((xy - x0) ** 2, axis=1)))
        st = O.knn(xy, [c], 37)[0]
        W, _ = O.stencil_weights(xy, st, c, m, l, [(O.DX, 0, 0)])
        errs.append(abs(np.dot(W[0], f(xy[st])) - exact))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(hs))
    assert np.all(slopes > l - 0.6) and np.all(slopes < l + 1.6), slopes


def test_singular_stencils_are_flagged():
    """Section 6.1: high degrees push Cartesian stencils to non-unisolvency.
    On the one-sided 37-node stencil of a Cartesian edge node the polynomial
    columns become dependent at degree 5 and 6 (flagged), not at degree 4;
    the symmetric interior stencil and the hexagonal one take degree 6. A
    duplicated node makes Phi singular."""
    nd = unit_square_cartesian(21)
    for c, l, expect in ((10, 4, 0), (10, 5, 1), (10, 6, 1), (10 * 21 + 10, 6, 0)):
        st = O.knn(nd.xy, [c], 37)[0]
        _, status = O.stencil_weights(nd.xy, st, c, 7, l, [(O.DX, 0, 0)])
        assert status == expect, (c, l)
    hexp = np.array([(i + 0.5 * (j % 2), j * math.sqrt(3) / 2) for j in range(15) for i in range(15)])
    c = 7 * 15 + 7
    st = O.knn(hexp, [c], 37)[0]
    _, status = O.stencil_weights(hexp, st, c, 7, 6, [(O.DX, 0, 0)])
    assert status == 0
    xy = nd.xy.copy()
    st = O.knn(xy, [10 * 21 + 10], 37)[0]
    xy[st[5]] = xy[st[6]]
    _, status = O.stencil_weights(xy, st, 10 * 21 + 10, 5, 4, [(O.DX, 0, 0)])
    assert status == 1
