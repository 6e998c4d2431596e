"""Collocation (CRVPINN) pressure operator, Gram matrix, robust loss (oracle).

Follows the CRVPINN section of the paper:
  * collocation grid Omega_h = {(ih, jh)}, h = 1/N (eq. 21), here in d = 2 or 3;
  * forward differences nabla_+ (eq. 22);
  * discrete products (u,v)_h = h^d sum u v and
    (u,v)_{nabla,h} = sum_dir (nabla_dir+ u, nabla_dir+ v)_h;
  * Kronecker-delta test functions (first eq. 23), nodal coefficient alpha and
    right-hand side (second eq. 23);
  * residual RES_kl = a_h(u, delta_kl) - (q, delta_kl)_h (eq. 24-25);
  * Gram matrix G = ((delta, delta))_{nabla,h} (eq. 26) and robust loss
    LOSS = RES^T G^{-1} RES (eq. 27-28).

Readings taken where the paper is silent or inconsistent:
  * sign: -div(alpha grad p) = q with q the total injection (q > 0 injects);
    with gravity q becomes q - div_+(g F) (gravity_divergence); a_h(u, v) = h^d sum over grid edges (p, p+e) of
    alpha_p nabla_e+ u(p) nabla_e+ v(p) (alpha taken at the edge's lower node);
  * tests delta_kl at interior nodes only, trial functions zero on the boundary;
  * G is built from the paper's own products, so it equals the integer
    5-point stencil in 2D (h * 7-point in 3D): the h^-2 printed in eq. 26 is
    not applied;
  * G^{-1} is applied exactly.  The oracle uses the orthonormal DST-I, which
    diagonalises G on the interior grid (a different algorithm from the HIP
    path, and pinned against a dense inverse on small grids).

Arrays are nodal with numpy shape (n,)*d, x the last (fastest) axis.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def relperm(s: np.ndarray, n: float):
    """Brooks-Corey relative permeabilities with zero residual saturation,
    evaluated at clamp(s, 0, 1): (kr_w, kr_g) = ((1-s)^n, s^n)."""
    sc = np.clip(s, 0.0, 1.0)
    return (1.0 - sc) ** n, sc ** n


def alpha_nodal(s_nodal, perm, mu_w, mu_g, n):
    """alpha = (kr_w/mu_w + kr_g/mu_g) K at the nodes (second eq. 23; the
    paper's linear S/mu is the case n = 1)."""
    krw, krg = relperm(s_nodal, n)
    return (krw / mu_w + krg / mu_g) * perm


def buoyancy_flux(s_nodal, perm, mu_w, mu_g, n, rho_w, rho_g):
    """F = K (lambda_w rho_w + lambda_g rho_g) at the nodes, lambda = kr / mu
    at clamp(s, 0, 1): the density-weighted mobility that gravity multiplies
    in the pressure equation (eq. 5)."""
    krw, krg = relperm(s_nodal, n)
    return perm * (krw / mu_w * rho_w + krg / mu_g * rho_g)


def gravity_divergence(s_nodal, perm, mu_w, mu_g, n, rho_w, rho_g, gravity):
    """div_+ (g K (lambda_w rho_w + lambda_g rho_g)) at the nodes: the gravity
    part of the collocation right-hand side (the RHS_ij formula of the
    CRVPINN section and of algorithm steps 2 and 6), forward difference
    (eq. 22).

    Reading: g = -gravity e_v with gravity >= 0 and e_v the last coordinate
    (y in 2D, z in 3D; numpy axis 0), i.e. gravity points down; the vector
    form (grad p - rho g) of eq. 1-2 is taken as the definition.  Nodes on
    the top face, where the forward difference does not exist, get zero
    (the residual uses interior nodes only)."""
    f = buoyancy_flux(s_nodal, perm, mu_w, mu_g, n, rho_w, rho_g)
    n_elem = f.shape[0] - 1
    out = np.zeros_like(f)
    out[:-1] = -gravity * (f[1:] - f[:-1]) * n_elem
    return out


def _diff_1d(n_elem: int):
    """1D forward difference on nodes 0..N: (N, N+1), rows i: (-1 at i, +1 at
    i+1)/h, and the selector of each edge's lower node."""
    n = n_elem + 1
    h = 1.0 / n_elem
    i = np.arange(n_elem)
    d = sp.csr_matrix((np.r_[-np.ones(n_elem), np.ones(n_elem)] / h,
                       (np.r_[i, i], np.r_[i, i + 1])), shape=(n_elem, n))
    s = sp.csr_matrix((np.ones(n_elem), (i, i)), shape=(n_elem, n))
    return d, s


def _axis_ops(n_elem: int, dim: int):
    """For every axis: forward difference D_a (edges x nodes) on the full grid
    and the lower-node selector S_a.  Axis order: x (fastest) first."""
    n = n_elem + 1
    d1, s1 = _diff_1d(n_elem)
    eye = sp.identity(n, format="csr")
    ops = []
    for a in range(dim):  # a = 0 -> x, 1 -> y, 2 -> z
        dk, sk = None, None
        for b in reversed(range(dim)):  # kron from the slowest axis to x
            fd = d1 if b == a else eye
            fs = s1 if b == a else eye
            dk = fd if dk is None else sp.kron(dk, fd, format="csr")
            sk = fs if sk is None else sp.kron(sk, fs, format="csr")
        ops.append((dk, sk))
    return ops


def interior_index(n_elem: int, dim: int) -> np.ndarray:
    n = n_elem + 1
    idx = np.arange(n ** dim).reshape((n,) * dim)
    sl = tuple(slice(1, n - 1) for _ in range(dim))
    return idx[sl].ravel()


def interior_mask(n_elem: int, dim: int) -> np.ndarray:
    n = n_elem + 1
    m = np.zeros((n,) * dim)
    m[tuple(slice(1, n - 1) for _ in range(dim))] = 1.0
    return m


def distance_factor(n_elem: int, dim: int) -> np.ndarray:
    """The distance form of the trial-function factor: prod over the axes of
    4 x_a (1 - x_a) at the nodes, x_a = i_a / N.  It vanishes on every
    boundary face (so the trial function meets the zero pressure condition,
    as with the interior indicator) and equals one at the centre."""
    x = np.arange(n_elem + 1) / n_elem
    f1 = 4.0 * x * (1.0 - x)
    out = f1
    for _ in range(dim - 1):
        out = np.multiply.outer(f1, out)
    return out


def stiffness_full(alpha: np.ndarray, n_elem: int) -> sp.csr_matrix:
    """Matrix of a_h on the full grid: a_h(u, v) = v^T A u with
    a_h(u,v) = h^d sum_a sum_edges alpha_lower (D_a u)(D_a v)."""
    dim = alpha.ndim
    h = 1.0 / n_elem
    a = None
    for d_a, s_a in _axis_ops(n_elem, dim):
        w = s_a @ alpha.ravel()
        term = d_a.T @ sp.diags(w) @ d_a
        a = term if a is None else a + term
    return (h ** dim) * a.tocsr()


def residual(u: np.ndarray, alpha: np.ndarray, q: np.ndarray) -> np.ndarray:
    """RES_k = a_h(u, delta_k) - (q, delta_k)_h for interior k (eq. 25);
    returns the interior array of shape (N-1,)*d."""
    dim = u.ndim
    n_elem = u.shape[0] - 1
    h = 1.0 / n_elem
    a = stiffness_full(alpha, n_elem)
    idx = interior_index(n_elem, dim)
    res = a[idx, :] @ u.ravel() - (h ** dim) * q.ravel()[idx]
    return res.reshape((n_elem - 1,) * dim)


def gram_matrix(n_elem: int, dim: int) -> sp.csr_matrix:
    """G_kl = (delta_k, delta_l)_{nabla,h} over interior nodes (eq. 26 from its
    defining inner product)."""
    ones = np.ones((n_elem + 1,) * dim)
    a = stiffness_full(ones, n_elem)
    idx = interior_index(n_elem, dim)
    return a[idx, :][:, idx].tocsr()


def gram_eigenvalues(n_elem: int, dim: int) -> np.ndarray:
    """Eigenvalues of G on the DST-I basis: h^(d-2) sum_a 4 sin^2(k_a pi / 2N),
    k_a = 1..N-1, shape (N-1,)*d."""
    m = n_elem - 1
    lam1 = 4.0 * np.sin(np.arange(1, m + 1) * np.pi / (2.0 * (m + 1))) ** 2
    grids = np.meshgrid(*([lam1] * dim), indexing="ij")
    return (1.0 / n_elem) ** (dim - 2) * sum(grids)


def gram_solve(res: np.ndarray) -> np.ndarray:
    """q = G^{-1} RES (eq. 28) by orthonormal DST-I diagonalisation."""
    dim = res.ndim
    n_elem = res.shape[0] + 1
    lam = gram_eigenvalues(n_elem, dim)
    rh = scipy.fft.dstn(res, type=1, norm="ortho")
    return scipy.fft.idstn(rh / lam, type=1, norm="ortho")


def loss(res: np.ndarray, q: np.ndarray) -> float:
    """LOSS = RES^T G^{-1} RES (eq. 27)."""
    return float(np.dot(res.ravel(), q.ravel()))


def grad_u(q: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """dLOSS/du on the full grid (before the boundary mask): 2 A^T q~ with q~
    the interior q extended by zero (G and A symmetric)."""
    dim = alpha.ndim
    n_elem = alpha.shape[0] - 1
    a = stiffness_full(alpha, n_elem)
    qt = np.zeros((n_elem + 1,) * dim)
    qt[tuple(slice(1, n_elem) for _ in range(dim))] = q
    return (2.0 * (a.T @ qt.ravel())).reshape(alpha.shape)


def grad_alpha(u: np.ndarray, q: np.ndarray) -> np.ndarray:
    """dLOSS/dalpha_p = 2 h^d sum_a [S_a^T ((D_a u)(D_a q~))]_p."""
    dim = u.ndim
    n_elem = u.shape[0] - 1
    h = 1.0 / n_elem
    qt = np.zeros_like(u)
    qt[tuple(slice(1, n_elem) for _ in range(dim))] = q
    g = np.zeros(u.size)
    for d_a, s_a in _axis_ops(n_elem, dim):
        g += s_a.T @ ((d_a @ u.ravel()) * (d_a @ qt.ravel()))
    return (2.0 * h ** dim * g).reshape(u.shape)


def direct_solve(alpha: np.ndarray, q: np.ndarray) -> np.ndarray:
    """u* with RES(u*) = 0, u* = 0 on the boundary: sparse direct (LU) solve of
    the same discrete pressure system the network is trained on.  This plays
    the role of the paper's direct-solver baseline."""
    dim = alpha.ndim
    n_elem = alpha.shape[0] - 1
    h = 1.0 / n_elem
    a = stiffness_full(alpha, n_elem)
    idx = interior_index(n_elem, dim)
    a_ii = a[idx, :][:, idx].tocsc()
    rhs = (h ** dim) * q.ravel()[idx]
    sol = spla.splu(a_ii).solve(rhs)
    u = np.zeros(alpha.size)
    u[idx] = sol
    return u.reshape(alpha.shape)


def grad_plus_norm(u: np.ndarray) -> np.ndarray:
    """|nabla_+ u| at every node where all forward differences exist."""
    dim = u.ndim
    n_elem = u.shape[0] - 1
    sl = tuple(slice(0, n_elem) for _ in range(dim))
    acc = np.zeros((n_elem,) * dim)
    for ax in range(dim):
        acc += (np.diff(u, axis=ax)[sl] * n_elem) ** 2
    return np.sqrt(acc)
