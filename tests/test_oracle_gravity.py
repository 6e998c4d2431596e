"""Pins of the oracle's gravity terms (pressure right-hand side of eq. 5 on the
collocation grid, gas flux of eq. 9-10), each against a value fixed by the
mathematics rather than by re-running the same formula:

* K linear in the vertical coordinate, uniform S: the divergence term is the
  constant -gravity (K' = 1) times the density-weighted mobility; K varying
  along x only gives zero (catches a wrong axis or sign);
* uniform K and S: no gravity source anywhere (hydrostatic balance of the
  discrete operator);
* the ADS right-hand side with uniform S, unit K and porosity, zero pressure
  and no wells equals S M 1 - tau lambda_g rho_g gravity (int B_x) x
  (B_v(1) - B_v(0)), written from the 1D mass matrices;
* the log K gradient with gravity on against central differences (2D, 3D);
* with gravity 0, nonzero densities change nothing in a coupled step.
"""
import numpy as np

from oracle import Oracle, ads, pressure
from paper_2604_20731_amd import inputs

G = dict(gravity=2.0, rho_w=1.2, rho_g=0.4)


def test_divergence_linear_perm_closed_form():
    ne = 8
    n = ne + 1
    y = np.arange(n) / ne
    for dim in (2, 3):
        shape = (n,) * dim
        perm = np.broadcast_to(1.0 + y.reshape((n,) + (1,) * (dim - 1)), shape).copy()
        for s_val, mob in ((0.0, 1.2 / 1.0), (1.0, 0.4 / 0.1)):
            s = np.full(shape, s_val)
            d = pressure.gravity_divergence(s, perm, 1.0, 0.1, 2.0, 1.2, 0.4, 2.0)
            inner = d[:-1]
            assert np.allclose(inner, -2.0 * mob, rtol=1e-12, atol=0), (dim, s_val)
            assert np.all(d[-1] == 0.0)
        # K varying along x only: no vertical change, no source
        x = np.arange(n) / ne
        perm_x = np.broadcast_to(1.0 + x, shape).copy()
        d = pressure.gravity_divergence(np.full(shape, 0.3), perm_x, 1.0, 0.1, 2.0, 1.2, 0.4, 2.0)
        assert np.all(d == 0.0)


def test_uniform_fields_have_no_gravity_source():
    shape = (9, 9)
    d = pressure.gravity_divergence(np.full(shape, 0.37), np.full(shape, 2.5), 1.0, 0.1, 2.0,
                                    1.2, 0.4, 9.81)
    assert np.all(d == 0.0)


def test_ads_gravity_term_closed_form():
    tau, s0 = 0.01, 0.3
    mu_g, n_exp, rho_g, grav = 0.1, 2.0, 0.4, 2.0
    for dim, ne, r in ((2, 6, 2), (3, 4, 2), (2, 5, 3)):
        sp = ads.Space(ne, r, dim)
        nb = sp.nb
        nodes = (ne + 1,) * dim
        s_coefs = np.full((nb,) * dim, s0)
        zero = np.zeros(nodes)
        b = ads.saturation_rhs(sp, s_coefs, np.zeros((nb,) * dim), np.ones(nodes),
                               np.ones(nodes), zero, zero, tau, 1.0, mu_g, n_exp, rho_g, grav)
        m = sp.m1.sum(axis=1)                      # int B_k over [0, 1]
        jump = np.zeros(nb)
        jump[-1], jump[0] = 1.0, -1.0               # B_k(1) - B_k(0)
        lam = s0 ** n_exp / mu_g
        horiz = m                                   # product of int B over the other axes
        for _ in range(dim - 2):
            horiz = np.multiply.outer(m, horiz)
        # numpy axis 0 is the vertical one
        expect = s0 * np.multiply.outer(m, horiz) \
            - tau * lam * rho_g * grav * np.multiply.outer(jump, horiz)
        assert np.allclose(b, expect, rtol=1e-12, atol=1e-15), (dim, ne, r)


def _grad_check(p, rng_seed):
    o = Oracle(p.dim, p.n_elem, p.degree, p.width, p.hidden, p.log_perm, p.porosity, p.wells,
               p.theta0, s0_coefs=np.random.default_rng(4).uniform(0, 0.6, (p.n_elem + p.degree,) * p.dim),
               **G)
    g = o.loss_grad_logperm()
    eps = 1e-6
    base = o.perm.copy()
    for k in np.random.default_rng(rng_seed).choice(base.size, size=12, replace=False):
        vals = []
        for sgn in (1, -1):
            lk = np.log(base).ravel().copy()
            lk[k] += sgn * eps
            o.perm = np.exp(lk).reshape(base.shape)
            o.refresh()
            vals.append(o.loss_and_grad()[0])
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(g.ravel()[k] - fd) < 1e-7 * max(1.0, abs(fd)), k
    o.perm = base
    o.refresh()
    # the gravity part is really there: without it the gradient differs
    o.gravity = 0.0
    o.refresh()
    assert np.max(np.abs(o.loss_grad_logperm() - g)) > 1e-6


def test_logperm_gradient_with_gravity_2d():
    _grad_check(inputs.make_problem("tiny"), 2)


def test_logperm_gradient_with_gravity_3d():
    wells = np.array([[0.5, 0.5, 1.0]])
    _grad_check(inputs.make_problem("c5", n_elem=4, width=8, hidden=2, wells=wells), 5)


def test_zero_gravity_ignores_densities():
    p = inputs.make_problem("tiny")
    a = Oracle(p.dim, p.n_elem, p.degree, p.width, p.hidden, p.log_perm, p.porosity, p.wells,
               p.theta0)
    b = Oracle(p.dim, p.n_elem, p.degree, p.width, p.hidden, p.log_perm, p.porosity, p.wells,
               p.theta0, gravity=0.0, rho_w=1.2, rho_g=0.4)
    for o in (a, b):
        o.pretrain(5)
        o.step(1e-4)
    assert np.array_equal(a.s, b.s) and np.array_equal(a.theta, b.theta)
