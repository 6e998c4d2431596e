"""B-spline space on an open uniform knot vector (oracle, test infrastructure).

Follows the discretisation section of the paper: the saturation and the
projected pressure are expanded in tensor products of 1D B-splines of order r
and continuity C^(r-1) (expansion of S_n, S_{n+1} and the test function v),
and the L2 mass matrix factorises as a Kronecker product of 1D mass matrices
(eq. 14).  Basis values come from the Cox-de Boor recursion written out here;
integrals use (r+1)-point Gauss-Legendre rules per element, which integrate the
degree-2r products of basis functions exactly.
"""
from __future__ import annotations

import numpy as np


def knot_vector(n_elem: int, r: int) -> np.ndarray:
    """Open uniform knots on [0,1]: r+1 zeros, the interior breakpoints e/Ne,
    r+1 ones; this gives Ne + r basis functions."""
    inner = np.arange(1, n_elem) / n_elem
    return np.concatenate([np.zeros(r + 1), inner, np.ones(r + 1)])


def n_basis(n_elem: int, r: int) -> int:
    return n_elem + r


def _safe_div(a, b):
    out = np.zeros(np.broadcast(a, b).shape)
    nz = b != 0
    np.divide(a, b, out=out, where=np.broadcast_to(nz, out.shape))
    return out


def basis(n_elem: int, r: int, x: np.ndarray, deriv: int = 0) -> np.ndarray:
    """Values (deriv=0) or first derivatives (deriv=1) of all Ne+r basis
    functions at points x; returns shape (len(x), Ne+r).

    Degree-0 functions are indicators of [t_i, t_{i+1}); the point x = 1 is
    assigned to the last non-empty span so the basis stays a partition of
    unity on the closed interval.
    """
    t = knot_vector(n_elem, r)
    x = np.asarray(x, dtype=np.float64)
    nk = len(t)
    b = np.zeros((len(x), nk - 1))
    for i in range(nk - 1):
        if t[i] < t[i + 1]:
            b[:, i] = (x >= t[i]) & (x < t[i + 1])
    last = np.max(np.nonzero(t[:-1] < t[1:])[0])
    b[x >= 1.0, :] = 0.0
    b[x >= 1.0, last] = 1.0
    for k in range(1, r + 1):
        nb = nk - 1 - k
        new = np.zeros((len(x), nb))
        dnew = np.zeros((len(x), nb))
        for i in range(nb):
            left = _safe_div(x - t[i], t[i + k] - t[i]) * b[:, i]
            right = _safe_div(t[i + k + 1] - x, t[i + k + 1] - t[i + 1]) * b[:, i + 1]
            new[:, i] = left + right
            if k == r and deriv == 1:
                dl = _safe_div(np.float64(k), t[i + k] - t[i]) * b[:, i]
                dr = _safe_div(np.float64(k), t[i + k + 1] - t[i + 1]) * b[:, i + 1]
                dnew[:, i] = dl - dr
        if k == r and deriv == 1:
            return dnew
        b = new
    if deriv == 1:  # r == 0
        return np.zeros_like(b)
    return b


def gauss_rule(n_elem: int, r: int):
    """(r+1)-point Gauss-Legendre rule on every element of [0,1]:
    points (Ne*(r+1),) and weights (same shape)."""
    xi, wi = np.polynomial.legendre.leggauss(r + 1)
    he = 1.0 / n_elem
    e = np.arange(n_elem)[:, None]
    xg = (e + 0.5 * (xi[None, :] + 1.0)) * he
    wg = np.broadcast_to(0.5 * wi[None, :] * he, xg.shape)
    return xg.ravel(), wg.ravel().copy()


def mass_1d(n_elem: int, r: int) -> np.ndarray:
    """M_ik = int_0^1 B_i B_k dx (eq. 14, one direction), by Gauss quadrature."""
    xg, wg = gauss_rule(n_elem, r)
    bg = basis(n_elem, r, xg)
    return bg.T @ (wg[:, None] * bg)


def hat(n_elem: int, x: np.ndarray) -> np.ndarray:
    """Piecewise-linear nodal (Q1 in 1D) hat functions of the nodes i/Ne at
    points x; shape (len(x), Ne+1)."""
    x = np.asarray(x, dtype=np.float64)
    nodes = np.arange(n_elem + 1)
    return np.maximum(0.0, 1.0 - np.abs(x[:, None] * n_elem - nodes[None, :]))


def node_points(n_elem: int) -> np.ndarray:
    return np.arange(n_elem + 1) / n_elem
