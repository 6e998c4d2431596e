"""Pins of the oracle's coupled algorithm on a tiny problem: the parameter
gradient against central finite differences of the robust loss (whole chain,
including the boundary mask), the loss against a dense Gram inverse, the
saturation mass balance over a coupled step, and basic algorithm invariants."""
import numpy as np

from oracle import Oracle, cfl_dt, pressure
from paper_2604_20731_amd import inputs


def _tiny(**kw):
    p = inputs.make_problem("tiny", **kw)
    return p, Oracle(p.dim, p.n_elem, p.degree, p.width, p.hidden, p.log_perm,
                     p.porosity, p.wells, p.theta0)


def test_theta_gradient_matches_central_differences():
    p, o = _tiny()
    th = o.theta + 0.05 * np.random.default_rng(0).standard_normal(o.theta.size)
    _, g = o.loss_and_grad(th)
    eps = 1e-6
    for k in np.random.default_rng(1).choice(th.size, size=20, replace=False):
        e = np.zeros_like(th); e[k] = eps
        fd = (o.loss_and_grad(th + e)[0] - o.loss_and_grad(th - e)[0]) / (2 * eps)
        assert abs(g[k] - fd) < 1e-7 * max(1.0, abs(fd)), k


def test_loss_equals_dense_gram_form():
    p, o = _tiny()
    u = o.u_nodal()
    res = pressure.residual(u, o.alpha, o.q)
    g = pressure.gram_matrix(p.n_elem, 2).toarray()
    dense = float(res.ravel() @ np.linalg.solve(g, res.ravel()))
    assert abs(o.loss_and_grad()[0] - dense) < 1e-12 * max(1, dense)


def test_logperm_gradient_matches_central_differences():
    p, o = _tiny()
    g = o.loss_grad_logperm()
    eps = 1e-6
    base = o.perm.copy()
    for k in np.random.default_rng(2).choice(base.size, size=10, replace=False):
        vals = []
        for sgn in (1, -1):
            lk = np.log(base).ravel().copy(); lk[k] += sgn * eps
            o.perm = np.exp(lk).reshape(base.shape)
            o.refresh()
            vals.append(o.loss_and_grad()[0])
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(g.ravel()[k] - fd) < 1e-7 * max(1.0, abs(fd))
    o.perm = base
    o.refresh()


def test_pretrain_and_step_invariants():
    wells = np.array([[0.375, 0.5, 1.0], [0.625, 0.375, 0.5]])
    p, o = _tiny(wells=wells)
    l0 = o.loss_and_grad()[0]
    o.pretrain(30)
    assert o.loss_history[0] == l0 and o.loss_history[-1] < l0
    dt = cfl_dt(o)
    assert dt > 0
    mass0 = float(np.sum(o.space.mass_full() @ o.s.ravel()))
    o.step(dt)
    u, s, sn = o.fields()
    mass1 = float(np.sum(o.space.mass_full() @ s.ravel()))
    # injectors only, uniform porosity 0.2: the gas volume grows by dt * sum(rate) / phi
    assert abs((mass1 - mass0) - dt * wells[:, 2].sum() / 0.2) < 1e-12
    assert np.all(u[0] == 0) and np.all(u[-1] == 0) and np.all(u[:, 0] == 0)
    assert s.shape == (p.n_elem + 2,) * 2 and sn.shape == (p.n_elem + 1,) * 2
    assert len(o.loss_history) == 30 + o.adam_iters


def _tiny3d():
    wells = np.array([[0.5, 0.5, 1.0]])
    p = inputs.make_problem("c5", n_elem=4, width=8, hidden=2, wells=wells)
    return p, Oracle(p.dim, p.n_elem, p.degree, p.width, p.hidden, p.log_perm,
                     p.porosity, p.wells, p.theta0)


def test_gradients_3d_match_central_differences():
    """3D (h L7 Gram, h-weighted stencil): dLOSS/dtheta and dLOSS/dlogK
    against central differences of the whole chain."""
    p, o = _tiny3d()
    th = o.theta + 0.05 * np.random.default_rng(3).standard_normal(o.theta.size)
    _, g = o.loss_and_grad(th)
    eps = 1e-6
    for k in np.random.default_rng(4).choice(th.size, size=12, replace=False):
        e = np.zeros_like(th); e[k] = eps
        fd = (o.loss_and_grad(th + e)[0] - o.loss_and_grad(th - e)[0]) / (2 * eps)
        assert abs(g[k] - fd) < 1e-7 * max(1.0, abs(fd)), k
    gl = o.loss_grad_logperm(th)
    base = o.perm.copy()
    for k in np.random.default_rng(5).choice(base.size, size=12, replace=False):
        vals = []
        for sgn in (1, -1):
            lk = np.log(base).ravel().copy(); lk[k] += sgn * eps
            o.perm = np.exp(lk).reshape(base.shape)
            o.refresh()
            vals.append(o.loss_and_grad(th)[0])
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(gl.ravel()[k] - fd) < 1e-7 * max(1.0, abs(fd)), k
    o.perm = base
    o.refresh()


def _tiny_factor(dim=2):
    p = (inputs.make_problem("tiny") if dim == 2 else
         inputs.make_problem("c5", n_elem=4, width=8, hidden=2, wells=np.array([[0.5, 0.5, 1.0]])))
    return p, Oracle(p.dim, p.n_elem, p.degree, p.width, p.hidden, p.log_perm,
                     p.porosity, p.wells, p.theta0, boundary_factor=1)


def test_distance_factor_trial_function_closed_form():
    """With every weight zero the network is its output bias b, so the trial
    function is b prod_a 4 x_a (1 - x_a), written out node by node here."""
    p, o = _tiny_factor()
    th = np.zeros_like(o.theta)
    th[-1] = 0.7
    u = o.u_nodal(th)
    n = p.n_elem
    for j in range(n + 1):
        for i in range(n + 1):
            x, y = i / n, j / n
            assert abs(u[j, i] - 0.7 * 16 * x * (1 - x) * y * (1 - y)) < 1e-15
    assert np.all(u[0] == 0) and np.all(u[-1] == 0) and np.all(u[:, 0] == 0)
    assert np.all(u[:, -1] == 0)


def test_distance_factor_gradients_match_central_differences():
    """dLOSS/dtheta with the distance factor (the backward must carry the
    factor, not the indicator), 2D and 3D, against central differences."""
    for dim, seed in ((2, 6), (3, 8)):
        p, o = _tiny_factor(dim)
        th = o.theta + 0.05 * np.random.default_rng(seed).standard_normal(o.theta.size)
        _, g = o.loss_and_grad(th)
        eps = 1e-6
        for k in np.random.default_rng(seed + 1).choice(th.size, size=12, replace=False):
            e = np.zeros_like(th); e[k] = eps
            fd = (o.loss_and_grad(th + e)[0] - o.loss_and_grad(th - e)[0]) / (2 * eps)
            assert abs(g[k] - fd) < 1e-7 * max(1.0, abs(fd)), (dim, k)
