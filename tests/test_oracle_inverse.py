"""Pins of the oracle's inverse-problem pieces (the paper's future work:
recovering reservoir parameters from observations), on a tiny problem:

* the objective LOSS + sum_p w_p (u_p - d_p)^2 against central finite
  differences in the network parameters and in the nodal log K (the misfit
  depends on log K only through the network, so the log K gradient is that of
  the robust loss);
* the misfit written out from its definition: zero weights change nothing,
  data equal to the network pressure add nothing, and shifting the data by a
  constant c moves the objective by c^2 sum w - 2c sum w (u - d);
* the joint Adam: the first log K step is -lr g / (|g| + eps) per node (bias
  corrections cancel at t = 1), and the iteration lowers the objective from
  a perturbed start."""
import numpy as np

from oracle import Oracle
from paper_2604_20731_amd import inputs


def _tiny(seed=0):
    p = inputs.make_problem("tiny", seed=seed)
    o = Oracle(p.dim, p.n_elem, p.degree, p.width, p.hidden, p.log_perm, p.porosity, p.wells,
               p.theta0)
    return p, o


def _observe(o, seed=3, every=2):
    """Data: the network pressure plus noise at every `every`-th interior node."""
    rng = np.random.default_rng(seed)
    u = o.u_nodal()
    w = np.zeros_like(u)
    w[1:-1:every, 1:-1:every] = 0.5
    d = u + 0.1 * rng.standard_normal(u.shape) * (w > 0)
    o.set_observations(d, w)
    return d, w


def test_objective_theta_gradient_with_misfit_matches_central_differences():
    p, o = _tiny()
    _observe(o)
    th = o.theta + 0.05 * np.random.default_rng(0).standard_normal(o.theta.size)
    _, g = o.loss_and_grad(th)
    eps = 1e-6
    for k in np.random.default_rng(1).choice(th.size, size=20, replace=False):
        e = np.zeros_like(th)
        e[k] = eps
        fd = (o.loss_and_grad(th + e)[0] - o.loss_and_grad(th - e)[0]) / (2 * eps)
        assert abs(g[k] - fd) < 1e-7 * max(1.0, abs(fd)), k


def test_objective_logperm_gradient_with_misfit_matches_central_differences():
    p, o = _tiny()
    _observe(o)
    lk = p.log_perm.copy()
    g = o.loss_grad_logperm()
    eps = 1e-6
    rng = np.random.default_rng(2)
    for _ in range(12):
        i, j = rng.integers(0, p.n_elem + 1, size=2)
        a = lk.copy()
        a[j, i] += eps
        o.set_log_perm(a)
        jp = o.loss_and_grad()[0]
        a[j, i] -= 2 * eps
        o.set_log_perm(a)
        jm = o.loss_and_grad()[0]
        o.set_log_perm(lk)
        fd = (jp - jm) / (2 * eps)
        assert abs(g[j, i] - fd) < 1e-7 * max(1.0, abs(fd)), (i, j)


def test_misfit_special_cases():
    p, o = _tiny()
    l0, g0 = o.loss_and_grad()
    u = o.u_nodal()
    o.set_observations(u + 1.0, np.zeros_like(u))        # zero weights
    l1, g1 = o.loss_and_grad()
    assert l1 == l0 and np.array_equal(g1, g0)
    w = np.zeros_like(u)
    w[1:-1, 1:-1] = 2.0
    o.set_observations(u, w)                             # data = the network's pressure
    l2, g2 = o.loss_and_grad()
    assert abs(l2 - l0) <= 1e-15 * abs(l0) and np.allclose(g2, g0, rtol=0, atol=1e-15)
    d = u + 0.3 * np.random.default_rng(5).standard_normal(u.shape)
    o.set_observations(d, w)
    la = o.loss_and_grad()[0]
    c = 0.25
    o.set_observations(d + c, w)
    lb = o.loss_and_grad()[0]
    expect = c * c * w.sum() - 2.0 * c * np.sum(w * (u - d))
    assert abs((lb - la) - expect) < 1e-12 * max(1.0, abs(expect))


def test_first_logperm_step_and_descent():
    """From the network trained at the true K, observed everywhere inside,
    and a perturbed log K: the first step is Adam's closed form, and the
    objective falls at every checkpoint (node-by-node log K with no prior is
    not identifiable, so the error of log K itself is not pinned)."""
    p, o = _tiny()
    o.train(200)
    d = o.u_nodal()
    w = np.zeros_like(d)
    w[1:-1, 1:-1] = 1.0
    o.set_observations(d, w)
    start = p.log_perm + 0.3 * np.random.default_rng(7).standard_normal(p.log_perm.shape)
    o.set_log_perm(start)
    g = o.loss_grad_logperm()
    j = [o.loss_and_grad()[0]]
    lr = 1e-2
    o.invert(1, lr)
    step = o.log_perm - start
    assert np.allclose(step, -lr * g / (np.abs(g) + o.adam.eps), rtol=1e-12, atol=1e-15)
    for _ in range(3):
        o.invert(100, lr)
        j.append(o.loss_and_grad()[0])
    assert all(b < a for a, b in zip(j, j[1:])), j
    assert j[-1] < 0.5 * j[0]
