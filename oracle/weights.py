"""RBF-FD weights from PHS + polynomials: one saddle-point solve per stencil.

Section 3, Eq. (weights): with phi(r) = r^m (m odd) and all bivariate monomials
p_q of degree <= l, the weights w of operator L at centre x_c solve

    [ Phi  P ] [w]   [ L phi(||x - x_j||) |_{x = x_c} ]
    [ P^T  0 ] [v] = [ L p_q |_{x = x_c}              ]

with Phi_jk = ||x_j - x_k||^m and P_jq = p_q(x_j); v is discarded. This
oracle computes that unique solution as accurately as it can:

1. the stencil is written in a local frame centred at x_c and scaled by
   rho = max_j ||x_j - x_c|| (the exact solution is invariant to this up to
   the factor rho^-q, q = derivative order; monomials are in graded order
   x^(d-b) z^b for d = 0..l, b = 0..d),
2. the system is formed in 64-bit-mantissa extended precision (x87 long
   double) from the FP64 node coordinates: for one-sided degree-5 stencils
   rounding the entries to FP64 alone moves the weights by ~5e-10,
3. LU with partial pivoting of the system rounded to FP64 (LAPACK getrf),
4. iterative refinement against the extended-precision system, residuals
   in extended precision, until the correction stops shrinking,
5. rescaling by rho^-q (extended precision), rounded to FP64 at the end.

Operator right-hand sides for phi = r^m (d = 2):
  Dx  : -m r^(m-2) x_j        (x_j, z_j: local offsets of node j)
  Dz  : -m r^(m-2) z_j
  Lap : m^2 r^(m-2)           (Eq. eqn:laplacian with d = 2)
  Lap^k: prod_{i<k} (m-2i)^2 r^(m-2k)   (Eq. eqn:laplacian applied k times;
                              continuous only for m >= 2k+1, Section 5.3)
  Dzz : m r^(m-2) + m(m-2) r^(m-4) z_j^2
  Dxx : m r^(m-2) + m(m-2) r^(m-4) x_j^2
and 0 at the centre node (r = 0) for every operator.
Polynomial rows hold L p_q at the centre: Lap^k(x^a z^b) at 0 is
C(k, a/2) a! b! when a + b = 2k with a, b even, else 0.

A stencil is reported singular (status 1) when the smallest |U_kk| of the
factorisation is below 1e-13 max|A| or refinement does not converge.
"""

import math
import numpy as np
import scipy.linalg

from .stencils import min_image

DX, DZ, LAP, HYPERLAP, DZZ, DXX = 1, 2, 3, 4, 5, 6


def poly_exponents(l: int):
    """Graded monomial exponents (a, b) of x^a z^b, degree <= l."""
    return [(d - b, b) for d in range(l + 1) for b in range(d + 1)]


def op_order(kind: int, k: int = 0) -> int:
    """Derivative order q of the operator (weights scale as rho^-q)."""
    return {DX: 1, DZ: 1, LAP: 2, DZZ: 2, DXX: 2, HYPERLAP: 2 * k}[kind]


def phs_apply(kind: int, m: int, k: int, x: np.ndarray, z: np.ndarray) -> np.ndarray:
    """L applied to ||x - x_j||^m as a function of x, evaluated at the centre
    (the origin of the local frame); (x, z) are the offsets of node j. The
    result has the floating type of (x, z) (FP64 or extended)."""
    x = np.asarray(x)
    z = np.asarray(z)
    if x.dtype.kind != "f":
        x = x.astype(np.float64)
        z = z.astype(np.float64)
    r = np.sqrt(x * x + z * z)
    out = np.zeros_like(r)
    nz = r > 0.0
    rn = r[nz]
    if kind == DX:
        out[nz] = -m * rn ** (m - 2) * x[nz]
    elif kind == DZ:
        out[nz] = -m * rn ** (m - 2) * z[nz]
    elif kind == LAP:
        out[nz] = m * m * rn ** (m - 2)
    elif kind == HYPERLAP:
        if m < 2 * k + 1:
            raise ValueError("Lap^k of r^m needs m >= 2k+1")
        c = 1.0
        for i in range(k):
            c *= float((m - 2 * i) ** 2)
        out[nz] = c * rn ** (m - 2 * k)
    elif kind == DZZ:
        out[nz] = m * rn ** (m - 2) + m * (m - 2) * rn ** (m - 4) * z[nz] ** 2
    elif kind == DXX:
        out[nz] = m * rn ** (m - 2) + m * (m - 2) * rn ** (m - 4) * x[nz] ** 2
    else:
        raise ValueError(kind)
    return out


def poly_apply(kind: int, k: int, a: int, b: int) -> float:
    """L(x^a z^b) evaluated at the origin."""
    if kind == DX:
        return 1.0 if (a, b) == (1, 0) else 0.0
    if kind == DZ:
        return 1.0 if (a, b) == (0, 1) else 0.0
    if kind == LAP:
        return 2.0 if (a, b) in ((2, 0), (0, 2)) else 0.0
    if kind == DZZ:
        return 2.0 if (a, b) == (0, 2) else 0.0
    if kind == DXX:
        return 2.0 if (a, b) == (2, 0) else 0.0
    if kind == HYPERLAP:
        if a + b != 2 * k or a % 2 or b % 2:
            return 0.0
        return float(math.comb(k, a // 2) * math.factorial(a) * math.factorial(b))
    raise ValueError(kind)


def local_frame(xy: np.ndarray, stencil: np.ndarray, center: int, period_x: float,
                dtype=np.float64):
    """Offsets of the stencil nodes from the centre (minimum image in x, the
    image chosen from the FP64 offset as in the stencil search), divided by
    rho = the largest offset length, all in ``dtype``. Returns (x, z, rho)."""
    d64 = xy[stencil, 0] - xy[center, 0]
    shift = np.where(d64 > 0.5 * period_x, -period_x, np.where(d64 < -0.5 * period_x, period_x, 0.0)) \
        if period_x > 0.0 else np.zeros_like(d64)
    X = xy.astype(dtype)
    dx = (X[stencil, 0] - X[center, 0]) + shift.astype(dtype)
    dz = X[stencil, 1] - X[center, 1]
    rho = np.sqrt(np.max(dx * dx + dz * dz))
    return dx / rho, dz / rho, rho


def saddle_matrix(x: np.ndarray, z: np.ndarray, m: int, l: int) -> np.ndarray:
    """[Phi P; P^T 0] of Eq. (weights) for local offsets (x, z)."""
    n = x.size
    exps = poly_exponents(l)
    M = len(exps)
    A = np.zeros((n + M, n + M), dtype=x.dtype)
    rx = x[:, None] - x[None, :]
    rz = z[:, None] - z[None, :]
    A[:n, :n] = np.sqrt(rx * rx + rz * rz) ** m
    for q, (a, b) in enumerate(exps):
        col = x ** a * z ** b
        A[:n, n + q] = col
        A[n + q, :n] = col
    return A


def saddle_rhs(x, z, m, l, ops):
    """Right-hand sides [L phi_j ; L p_q] for each (kind, k) in ops."""
    n = x.size
    exps = poly_exponents(l)
    B = np.zeros((n + len(exps), len(ops)), dtype=x.dtype)
    for c, (kind, k) in enumerate(ops):
        B[:n, c] = phs_apply(kind, m, k, x, z)
        B[n:, c] = [poly_apply(kind, k, a, b) for (a, b) in exps]
    return B


def refined_solve(A: np.ndarray, B: np.ndarray, max_iter: int = 10):
    """LU with partial pivoting of A rounded to FP64 + iterative refinement
    against A and B as given (extended precision). Returns (X extended,
    status)."""
    A64 = A.astype(np.float64)
    lu, piv = scipy.linalg.lu_factor(A64, check_finite=True)
    status = 0
    if np.min(np.abs(np.diag(lu))) < 1e-13 * np.max(np.abs(A64)):
        status = 1
    X = scipy.linalg.lu_solve((lu, piv), B.astype(np.float64))
    AL = A.astype(np.longdouble)
    BL = B.astype(np.longdouble)
    XL = X.astype(np.longdouble)
    prev = np.inf
    converged = False
    for _ in range(max_iter):
        R = BL - AL @ XL
        D = scipy.linalg.lu_solve((lu, piv), R.astype(np.float64))
        XL = XL + D.astype(np.longdouble)
        size = float(np.max(np.abs(D)))
        scale = float(np.max(np.abs(XL)))
        if size <= 2.0 ** -62 * scale:
            converged = True
            break
        if size >= 0.5 * prev:          # stagnation: no further gain
            converged = size <= 1e-6 * scale
            break
        prev = size
    if not converged or not np.all(np.isfinite(XL)):
        status = 1
    return XL, status


def stencil_weights(xy, stencil, center, m, l, ops, period_x=0.0):
    """Weights of every operator at one centre.

    ops: list of (kind, k, phs_order) with phs_order 0 meaning m, and for
    Lap^k, k = 0 meaning the largest power the PHS order allows, (m-1)/2
    (Section 5.3: continuity needs m >= 2k+1). Operators sharing a PHS order
    share one solve. Returns (w [len(ops)][n], status)."""
    x, z, rho = local_frame(np.asarray(xy, np.float64), np.asarray(stencil), center, period_x,
                            dtype=np.longdouble)
    n = x.size
    W = np.zeros((len(ops), n))
    status = 0
    groups = {}
    resolved = []
    for i, (kind, k, mo) in enumerate(ops):
        mm = mo if mo else m
        if kind == HYPERLAP and k == 0:
            k = (mm - 1) // 2
        resolved.append((kind, k, mm))
        groups.setdefault(mm, []).append(i)
    ops = resolved
    for mm, members in groups.items():
        A = saddle_matrix(x, z, mm, l)
        B = saddle_rhs(x, z, mm, l, [(ops[i][0], ops[i][1]) for i in members])
        X, st = refined_solve(A, B)
        status |= st
        for c, i in enumerate(members):
            kind, k, _ = ops[i]
            W[i] = (X[:n, c] / rho ** op_order(kind, k)).astype(np.float64)
    return W, status


def all_weights(xy, idx, centers, m, l, ops, period_x=0.0, n_per=None, m_per=None, l_per=None):
    """Weights for many centres: idx[a][:n_a] is the stencil of centers[a].
    Returns (w [len(ops)][len(centers)][n_max] zero-padded, status [len])."""
    idx = np.asarray(idx)
    nc, n_max = idx.shape
    W = np.zeros((len(ops), nc, n_max))
    status = np.zeros(nc, np.int32)
    for a in range(nc):
        na = int(n_per[a]) if n_per is not None else n_max
        ma = int(m_per[a]) if m_per is not None else m
        la = int(l_per[a]) if l_per is not None else l
        w, st = stencil_weights(xy, idx[a, :na], int(centers[a]), ma, la, ops, period_x)
        W[:, a, :na] = w
        status[a] = st
    return W, status
