"""IGA Galerkin pressure system (oracle, test infrastructure): the paper's
direct-solver path, which CRVPINN replaces (eq. 15-20).

    S P = F,   S_(kl),(mn) = int alpha grad B_kl . grad B_mn,
               F_kl = int q B_kl + int (g F_b) . grad B_kl,

with alpha = K (kr_w/mu_w + kr_g/mu_g)(S) and the buoyancy flux
F_b = K (kr_w rho_w/mu_w + kr_g rho_g/mu_g)(S), both at the Gauss points, and
P the B-spline coefficients of the pressure.  Solved here by a sparse direct
factorisation (the role MUMPS plays in the paper).

Readings:
  * sign: the weak form of eq. 5 under -div(alpha grad p) = q - div(g F_b)
    (the same reading as the collocation path) gives +(q, v) + (g F_b, grad v);
    eq. 15 prints -(q, v), which does not follow from eq. 5;
  * g = -gravity e_v (e_v the last coordinate), as in the collocation path;
  * p = 0 on the boundary: the B-spline coefficients on the boundary faces
    (first and last along every axis of an open knot vector) are fixed at 0
    and the system is solved for the others;
  * K and the well sources are nodal data, Q1-interpolated to the Gauss
    points; S is the spline; (r+1)^d Gauss points per element (as in the
    saturation update).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import pressure
from .ads import Space


def _gauss_op(space: Space, deriv_axis: int = -1) -> sp.csr_matrix:
    """Matrix from coefficients (C order, x fastest) to values at the Gauss
    points (same order): the Kronecker product of the 1D basis (or, along
    deriv_axis, derivative) tables."""
    mats = [space.dbg if a == deriv_axis else space.bg for a in range(space.dim)]
    out = None
    for a in reversed(range(space.dim)):  # slowest axis first in the Kronecker product
        m = sp.csr_matrix(mats[a])
        out = m if out is None else sp.kron(out, m, format="csr")
    return out


def _weights(space: Space) -> np.ndarray:
    w = space.wg
    out = w
    for _ in range(space.dim - 1):
        out = np.multiply.outer(w, out)
    return out.ravel()


def stiffness(space: Space, alpha_g: np.ndarray) -> sp.csr_matrix:
    """S = sum_a G_a^T diag(w alpha) G_a (eq. 18)."""
    w = _weights(space) * alpha_g.ravel()
    s = None
    for a in range(space.dim):
        g = _gauss_op(space, a)
        t = g.T @ sp.diags(w) @ g
        s = t if s is None else s + t
    return s.tocsr()


def load(space: Space, q_g: np.ndarray, flux_g=None, gravity: float = 0.0) -> np.ndarray:
    """F_k = int q B_k + int (g F_b) . grad B_k with g = -gravity e_v (eq. 20)."""
    f = space.integrate(q_g)
    if flux_g is not None and gravity != 0.0:
        f = f - gravity * space.integrate(flux_g, deriv_axis=space.dim - 1)
    return f


def interior_mask(space: Space) -> np.ndarray:
    """True for the coefficients not on a boundary face."""
    nb = space.nb
    m = np.zeros((nb,) * space.dim, dtype=bool)
    m[tuple(slice(1, nb - 1) for _ in range(space.dim))] = True
    return m


def solve(space: Space, alpha_g: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Coefficients P with S P = F on the interior coefficients, 0 on the
    boundary faces (sparse LU)."""
    s = stiffness(space, alpha_g)
    m = interior_mask(space).ravel()
    idx = np.nonzero(m)[0]
    sol = spla.splu(s[idx, :][:, idx].tocsc()).solve(f.ravel()[idx])
    out = np.zeros(m.size)
    out[idx] = sol
    return out.reshape((space.nb,) * space.dim)


def apply_stiffness(space: Space, alpha_g: np.ndarray, coefs: np.ndarray,
                    absolute: bool = False) -> np.ndarray:
    """S P in 2D without assembling S, one axis at a time (eq. 18):
        S P = B^T (c * (B P D^T)) D + D^T (c * (D P B^T)) B,
    B, D the 1D basis and derivative tables at the Gauss points, c = w alpha
    (arrays y-major, x fastest).  absolute: the same with |B|, |D| and |P|,
    an entrywise upper bound of |S| |P| (c > 0), for backward errors at sizes
    where the assembled S does not fit."""
    assert space.dim == 2
    b, d, p = space.bg, space.dbg, np.asarray(coefs).reshape(space.nb, space.nb)
    if absolute:
        b, d, p = np.abs(b), np.abs(d), np.abs(p)
    b, d = sp.csr_matrix(b), sp.csr_matrix(d)  # r+1 entries per row
    c = np.multiply.outer(space.wg, space.wg) * alpha_g.reshape(len(space.wg), len(space.wg))

    def term(ty, tx):  # ty^T (c * (ty P tx^T)) tx
        g = np.asarray(tx @ np.asarray(ty @ p).T).T
        return np.asarray(tx.T @ np.asarray(ty.T @ (c * g)).T).T

    return term(b, d) + term(d, b)


def fields_at_gauss(space: Space, s_coefs, perm, mu_w, mu_g, n_exp, rho_w=0.0, rho_g=0.0):
    """alpha and the buoyancy flux at the Gauss points from the saturation
    spline and the Q1-interpolated nodal permeability."""
    s = space.at_gauss(s_coefs)
    kg = space.nodal_at_gauss(perm)
    krw, krg = pressure.relperm(s, n_exp)
    alpha = kg * (krw / mu_w + krg / mu_g)
    flux = kg * (krw * rho_w / mu_w + krg * rho_g / mu_g)
    return alpha, flux


def pressure_solve(space: Space, s_coefs, perm, q_nodal, mu_w, mu_g, n_exp, gravity=0.0,
                   rho_w=0.0, rho_g=0.0) -> np.ndarray:
    """The Galerkin pressure of the current saturation (eq. 15-20)."""
    alpha, flux = fields_at_gauss(space, s_coefs, perm, mu_w, mu_g, n_exp, rho_w, rho_g)
    f = load(space, space.nodal_at_gauss(q_nodal), flux, gravity)
    return solve(space, alpha, f)
