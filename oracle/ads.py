"""IGA-ADS pieces: L2 projection, Kronecker mass solve, explicit saturation
substep (oracle, test infrastructure).

Follows the weak form of the saturation update (eq. 7-10, first use), its
B-spline Galerkin form (eq. 10-13, second use) and the Kronecker structure of
the mass matrix (eq. 14), and step 4 of the IGA-ADS-CRVPINN algorithm
(projection of the nodal network pressure into the B-spline space).

Readings taken where the paper is silent:
  * every integral uses (r+1)^d Gauss-Legendre points per element;
  * K, phi and the well sources are nodal data; at Gauss points they are the
    piecewise multilinear (Q1) interpolants of the nodal arrays;
  * the projected pressure is the L2 projection of the Q1 interpolant of the
    nodal network values (nodes = element vertices);
  * the boundary term is dropped (natural, no-flux saturation boundary), so
    the saturation mass changes only through the sources; S is never clipped,
    only the mobility arguments are clamped to [0, 1];
  * gas mobility lambda_g = kr_g(S)/mu_g with Brooks-Corey kr_g = s^n; the
    gas source is the well rate at injectors and f_g(S) = lambda_g/lambda_t
    times the rate at producers;
  * phi^-1 sits inside the integral (identical for uniform porosity).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import bspline


def along(mat: np.ndarray, arr: np.ndarray, axis: int) -> np.ndarray:
    """Apply mat (out x in) to one axis of arr."""
    return np.moveaxis(np.tensordot(mat, arr, axes=([1], [axis])), 0, axis)


def _axes(dim):
    """numpy axes of x, y[, z] for arrays shaped (..., y, x)."""
    return [dim - 1 - a for a in range(dim)]


class Space:
    """Tabulated 1D B-spline and hat data for one (Ne, r)."""

    def __init__(self, n_elem: int, r: int, dim: int):
        self.n_elem, self.r, self.dim = n_elem, r, dim
        self.nb = bspline.n_basis(n_elem, r)
        self.xg, self.wg = bspline.gauss_rule(n_elem, r)
        self.bg = bspline.basis(n_elem, r, self.xg)              # gauss x nb
        self.dbg = bspline.basis(n_elem, r, self.xg, deriv=1)    # gauss x nb
        self.hg = bspline.hat(n_elem, self.xg)                   # gauss x nodes
        self.bnode = bspline.basis(n_elem, r, bspline.node_points(n_elem))  # nodes x nb
        self.m1 = bspline.mass_1d(n_elem, r)
        self.m1_inv = np.linalg.inv(self.m1)

    # --- evaluation at Gauss points -------------------------------------
    def at_gauss(self, coefs: np.ndarray, deriv_axis: int = -1) -> np.ndarray:
        out = coefs
        for a, ax in enumerate(_axes(self.dim)):
            out = along(self.dbg if a == deriv_axis else self.bg, out, ax)
        return out

    def nodal_at_gauss(self, nodal: np.ndarray) -> np.ndarray:
        out = nodal
        for ax in _axes(self.dim):
            out = along(self.hg, out, ax)
        return out

    def at_nodes(self, coefs: np.ndarray) -> np.ndarray:
        """Spline values at the collocation nodes (= knots)."""
        out = coefs
        for ax in _axes(self.dim):
            out = along(self.bnode, out, ax)
        return out

    # --- integration against the basis -----------------------------------
    def integrate(self, vals_g: np.ndarray, deriv_axis: int = -1) -> np.ndarray:
        """b_k = sum_gauss w_g vals(g) B_k(g) (or d/dx_a B_k for a = deriv_axis)."""
        out = vals_g
        for a, ax in enumerate(_axes(self.dim)):
            tab = self.dbg if a == deriv_axis else self.bg
            out = along((tab * self.wg[:, None]).T, out, ax)
        return out

    # --- mass solves ------------------------------------------------------
    def mass_solve(self, b: np.ndarray) -> np.ndarray:
        """c = (M^x (x) M^y [(x) M^z])^{-1} b one direction at a time with the
        dense inverse of the 1D mass matrix (eq. 14)."""
        out = b
        for ax in _axes(self.dim):
            out = along(self.m1_inv, out, ax)
        return out

    def mass_solve_banded(self, b: np.ndarray) -> np.ndarray:
        """Same product, each direction by a banded Cholesky solve (LAPACK)."""
        r = self.r
        ab = np.zeros((r + 1, self.nb))
        for k in range(r + 1):
            ab[r - k, k:] = np.diagonal(self.m1, k)
        fac = scipy.linalg.cholesky_banded(ab)
        out = b
        for ax in _axes(self.dim):
            moved = np.moveaxis(out, ax, 0)
            sh = moved.shape
            sol = scipy.linalg.cho_solve_banded((fac, False), moved.reshape(sh[0], -1))
            out = np.moveaxis(sol.reshape(sh), 0, ax)
        return out

    def mass_full(self) -> np.ndarray:
        """The literal Kronecker mass matrix in the C order of the coefficient
        array (x fastest): M = M^(slowest) (x) ... (x) M^x."""
        m = self.m1
        for _ in range(self.dim - 1):
            m = np.kron(self.m1, m)
        return m

    def mass_solve_dense_kron(self, b: np.ndarray) -> np.ndarray:
        return np.linalg.solve(self.mass_full(), b.ravel()).reshape(b.shape)


def project_nodal(space: Space, u_nodal: np.ndarray) -> np.ndarray:
    """p with M p = b, b_k = int I_h(u) B_k (algorithm step 4)."""
    return space.mass_solve(space.integrate(space.nodal_at_gauss(u_nodal)))


def saturation_rhs(space: Space, s_coefs, p_coefs, perm, poro, q_inj, q_prod,
                   tau, mu_w, mu_g, n_exp, rho_g=0.0, gravity=0.0):
    """b_k = int [S B_k + tau phi^-1 (-lambda_g(S) K (grad p - rho_g g) . grad B_k
    + q_g B_k)] (eq. 9-10: the weak form of the explicit gas update, boundary
    term dropped as in eq. 9).

    Reading: g = -gravity e_v with e_v the last coordinate (y in 2D, z in
    3D), so only the vertical derivative changes: d_v p -> d_v p + rho_g
    gravity.  (Eq. 10 writes the term as rho_g g v_y, i.e. with g the signed
    vertical component; with g = -gravity the two agree.)"""
    dim = space.dim
    s = space.at_gauss(s_coefs)
    kg = space.nodal_at_gauss(perm)
    phig = space.nodal_at_gauss(poro)
    qig = space.nodal_at_gauss(q_inj)
    qpg = space.nodal_at_gauss(q_prod)
    sc = np.clip(s, 0.0, 1.0)
    lam_g = sc ** n_exp / mu_g
    lam_w = (1.0 - sc) ** n_exp / mu_w
    f_g = lam_g / (lam_g + lam_w)
    qg = qig + f_g * qpg
    b = space.integrate(s + tau * qg / phig)
    for a in range(dim):
        dp = space.at_gauss(p_coefs, deriv_axis=a)
        if a == dim - 1:
            dp = dp + rho_g * gravity
        flux = -tau / phig * lam_g * kg * dp
        b = b + space.integrate(flux, deriv_axis=a)
    return b


def saturation_substep(space: Space, s_coefs, p_coefs, perm, poro, q_inj, q_prod,
                       tau, mu_w, mu_g, n_exp, rho_g=0.0, gravity=0.0):
    """S^{n+1} = M^{-1} b (eq. 6 as the L2 projection of eq. 10-12)."""
    b = saturation_rhs(space, s_coefs, p_coefs, perm, poro, q_inj, q_prod,
                       tau, mu_w, mu_g, n_exp, rho_g, gravity)
    return space.mass_solve(b)
