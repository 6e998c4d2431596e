"""Pins of the oracle's collocation operator, Gram inverse, loss and gradients:
brute force on tiny grids, closed forms, manufactured solutions, invariants
and central finite differences."""
import itertools

import numpy as np
import pytest

from oracle import pressure


def _brute_ah(u, v, alpha):
    """a_h(u,v) = h^d sum over grid edges (p, p+e) of alpha_p (u(p+e)-u(p))/h * (v(p+e)-v(p))/h,
    by an explicit loop over every node and direction."""
    dim = u.ndim
    ne = u.shape[0] - 1
    h = 1.0 / ne
    tot = 0.0
    for p in itertools.product(range(ne + 1), repeat=dim):
        for a in range(dim):
            q = list(p)
            q[dim - 1 - a] += 1          # axis a = 0 is x, the last numpy axis
            if q[dim - 1 - a] > ne:
                continue
            q = tuple(q)
            tot += alpha[p] * (u[q] - u[p]) / h * (v[q] - v[p]) / h
    return h ** dim * tot


@pytest.mark.parametrize("dim", [2, 3])
def test_stiffness_matches_brute_force_bilinear_form(dim):
    ne = 4 if dim == 2 else 3
    rng = np.random.default_rng(0)
    alpha = rng.uniform(0.5, 2.0, size=(ne + 1,) * dim)
    a = pressure.stiffness_full(alpha, ne).toarray()
    n = (ne + 1) ** dim
    for i in range(n):
        for j in range(i, n):
            ei = np.zeros(n); ei[i] = 1
            ej = np.zeros(n); ej[j] = 1
            bf = _brute_ah(ei.reshape(alpha.shape), ej.reshape(alpha.shape), alpha)
            assert abs(a[j, i] - bf) < 1e-12 and abs(a[i, j] - bf) < 1e-12


def test_residual_explicit_stencil_2d():
    # RES_p = sum_dir [alpha_{p-e}(u_p - u_{p-e}) - alpha_p(u_{p+e} - u_p)] - h^2 q_p
    ne = 6
    h = 1.0 / ne
    rng = np.random.default_rng(1)
    alpha = rng.uniform(0.5, 2.0, size=(ne + 1, ne + 1))
    u = rng.standard_normal((ne + 1, ne + 1))
    q = rng.standard_normal((ne + 1, ne + 1))
    res = pressure.residual(u, alpha, q)
    for j in range(1, ne):
        for i in range(1, ne):
            s = (alpha[j, i - 1] * (u[j, i] - u[j, i - 1]) - alpha[j, i] * (u[j, i + 1] - u[j, i])
                 + alpha[j - 1, i] * (u[j, i] - u[j - 1, i]) - alpha[j, i] * (u[j + 1, i] - u[j, i])
                 - h * h * q[j, i])
            assert abs(res[j - 1, i - 1] - s) < 1e-12


def test_gram_is_integer_five_point_stencil_2d():
    ne = 5
    m = ne - 1
    g = pressure.gram_matrix(ne, 2).toarray()
    t = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    l5 = np.kron(t, np.eye(m)) + np.kron(np.eye(m), t)
    assert np.allclose(g, l5, atol=1e-13)
    assert np.allclose(np.diag(g), 4.0)


def test_gram_is_h_times_seven_point_stencil_3d():
    ne = 4
    m = ne - 1
    g = pressure.gram_matrix(ne, 3).toarray()
    t = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    i = np.eye(m)
    l7 = np.kron(np.kron(t, i), i) + np.kron(np.kron(i, t), i) + np.kron(np.kron(i, i), t)
    assert np.allclose(g, l7 / ne, atol=1e-13)


@pytest.mark.parametrize("dim,ne", [(2, 8), (2, 13), (3, 6)])
def test_gram_solve_equals_dense_inverse(dim, ne):
    rng = np.random.default_rng(2)
    res = rng.standard_normal((ne - 1,) * dim)
    g = pressure.gram_matrix(ne, dim).toarray()
    ref = np.linalg.solve(g, res.ravel()).reshape(res.shape)
    assert np.allclose(pressure.gram_solve(res), ref, atol=1e-11)


def _energy_seminorm2(e):
    dim = e.ndim
    ne = e.shape[0] - 1
    return float(e.ravel() @ (pressure.stiffness_full(np.ones_like(e), ne) @ e.ravel()))


def test_loss_identity_alpha_one_and_inf_sup_bounds():
    ne = 12
    rng = np.random.default_rng(3)
    mask = pressure.interior_mask(ne, 2)
    q = rng.standard_normal((ne + 1, ne + 1))
    u = rng.standard_normal((ne + 1, ne + 1)) * mask
    ones = np.ones_like(u)
    ustar = pressure.direct_solve(ones, q)
    res = pressure.residual(u, ones, q)
    lval = pressure.loss(res, pressure.gram_solve(res))
    assert abs(lval - _energy_seminorm2(u - ustar)) < 1e-10 * max(1.0, lval)
    # variable coefficient: alpha_min^2 <= LOSS / |u-u*|^2 <= alpha_max^2
    alpha = rng.uniform(0.3, 3.0, size=u.shape)
    ustar = pressure.direct_solve(alpha, q)
    res = pressure.residual(u, alpha, q)
    ratio = pressure.loss(res, pressure.gram_solve(res)) / _energy_seminorm2(u - ustar)
    assert alpha.min() ** 2 * (1 - 1e-12) <= ratio <= alpha.max() ** 2 * (1 + 1e-12)


def test_discrete_manufactured_solution_is_exact():
    ne = 10
    rng = np.random.default_rng(4)
    alpha = rng.uniform(0.5, 2.0, size=(ne + 1, ne + 1))
    u = rng.standard_normal((ne + 1, ne + 1)) * pressure.interior_mask(ne, 2)
    a = pressure.stiffness_full(alpha, ne)
    q = (a @ u.ravel()).reshape(u.shape) * ne ** 2      # (q, delta)_h = h^2 q
    assert np.max(np.abs(pressure.residual(u, alpha, q))) < 1e-12
    assert np.max(np.abs(pressure.direct_solve(alpha, q) - u)) < 1e-10


@pytest.mark.parametrize("variable", [False, True])
def test_continuum_manufactured_solution_order(variable):
    # -div(alpha grad p) = f, p = sin(pi x) sin(pi y)
    errs = []
    for ne in (16, 32, 64):
        x = np.arange(ne + 1) / ne
        xx, yy = np.meshgrid(x, x, indexing="xy")
        p = np.sin(np.pi * xx) * np.sin(np.pi * yy)
        if variable:
            al = 1.0 + 0.5 * xx * yy
            ax, ay = 0.5 * yy, 0.5 * xx
        else:
            al, ax, ay = np.ones_like(xx), 0.0, 0.0
        px = np.pi * np.cos(np.pi * xx) * np.sin(np.pi * yy)
        py = np.pi * np.sin(np.pi * xx) * np.cos(np.pi * yy)
        f = al * 2 * np.pi ** 2 * p - ax * px - ay * py
        u = pressure.direct_solve(al, f)
        errs.append(np.max(np.abs(u - p)))
    order = np.log2(errs[1] / errs[2])
    if variable:
        assert order > 0.9
    else:
        assert 1.9 < order < 2.1


def test_grad_u_and_grad_alpha_match_central_differences():
    ne = 6
    rng = np.random.default_rng(5)
    alpha = rng.uniform(0.5, 2.0, size=(ne + 1, ne + 1))
    q = rng.standard_normal((ne + 1, ne + 1))
    u = rng.standard_normal((ne + 1, ne + 1))

    def lfun(uu, aa):
        r = pressure.residual(uu, aa, q)
        return pressure.loss(r, pressure.gram_solve(r))

    res = pressure.residual(u, alpha, q)
    qq = pressure.gram_solve(res)
    gu = pressure.grad_u(qq, alpha)
    ga = pressure.grad_alpha(u, qq)
    eps = 1e-6
    for k in rng.choice((ne + 1) ** 2, size=12, replace=False):
        e = np.zeros(u.size); e[k] = eps
        e = e.reshape(u.shape)
        fd_u = (lfun(u + e, alpha) - lfun(u - e, alpha)) / (2 * eps)
        fd_a = (lfun(u, alpha + e) - lfun(u, alpha - e)) / (2 * eps)
        mask = pressure.interior_mask(ne, 2).ravel()[k]
        if mask:
            assert abs(gu.ravel()[k] - fd_u) < 1e-6 * max(1, abs(fd_u))
        assert abs(ga.ravel()[k] - fd_a) < 1e-6 * max(1, abs(fd_a))


def test_relperm_and_alpha():
    s = np.array([-0.5, 0.0, 0.25, 1.0, 1.5])
    krw, krg = pressure.relperm(s, 2.0)
    assert np.allclose(krw, [1, 1, 0.5625, 0, 0]) and np.allclose(krg, [0, 0, 0.0625, 1, 1])
    a = pressure.alpha_nodal(np.array([0.0, 1.0]), np.array([2.0, 3.0]), 1.0, 0.1, 2.0)
    assert np.allclose(a, [2.0, 30.0])
