"""Pins of the oracle's IGA Galerkin pressure system (eq. 15-20), each
against what the mathematics fixes:

* a pressure inside the spline space is reproduced exactly: with alpha = 1
  and q = -Lap p for p = x(1-x)y(1-y) (3D: also z(1-z)), given exactly at the
  Gauss points, Galerkin orthogonality makes the discrete solution p itself
  (2D quadratic and cubic, 3D quadratic);
* the interior system is symmetric positive definite;
* gravity enters only through the load: for F_b = rho_w K with K = 1 + y the
  gravity load -g int F_b d_y v equals the source g rho_w int v (integration
  by parts, v = 0 on the boundary), so both give the same pressure; a
  constant F_b gives no load on the interior coefficients;
* the whole path (fields from S and nodal K, sources from the nodes) leaves
  a residual of round-off size in the assembled interior system;
* the axis-by-axis product S P equals the assembled S times P, and its
  absolute form bounds |S| |P| entrywise.
"""
import numpy as np

from oracle import galerkin
from oracle.ads import Space


def _coords(space):
    xg = space.xg
    return np.meshgrid(*([xg] * space.dim), indexing="ij")  # axis 0 is the last coordinate


def test_polynomial_pressure_reproduced_exactly():
    for dim, ne, r in ((2, 6, 2), (2, 5, 3), (3, 4, 2)):
        sp = Space(ne, r, dim)
        c = _coords(sp)                        # c[0] = v (y or z), c[-1] = x
        bub = [t * (1 - t) for t in c]
        p_exact = np.prod(bub, axis=0)
        lap = np.zeros_like(p_exact)
        for a in range(dim):
            others = np.prod([bub[b] for b in range(dim) if b != a], axis=0)
            lap += -2.0 * others
        q = -lap
        alpha = np.ones_like(p_exact)
        coef = galerkin.solve(sp, alpha, galerkin.load(sp, q))
        assert np.allclose(sp.at_gauss(coef), p_exact, rtol=0, atol=1e-13), (dim, ne, r)


def test_interior_system_spd():
    sp = Space(6, 2, 2)
    rng = np.random.default_rng(0)
    alpha = np.exp(rng.standard_normal((sp.xg.size,) * 2))
    s = galerkin.stiffness(sp, alpha).toarray()
    idx = np.nonzero(galerkin.interior_mask(sp).ravel())[0]
    si = s[np.ix_(idx, idx)]
    assert np.allclose(si, si.T, rtol=0, atol=1e-14)
    assert np.linalg.eigvalsh(si).min() > 0


def test_gravity_load_equals_source_for_linear_flux():
    grav, rho_w = 3.0, 1.2
    for dim, ne, r in ((2, 6, 2), (3, 4, 2)):
        sp = Space(ne, r, dim)
        c = _coords(sp)
        kk = 1.0 + c[0]                        # K linear in the vertical coordinate
        zero = np.zeros_like(kk)
        p1 = galerkin.solve(sp, kk, galerkin.load(sp, zero, rho_w * kk, grav))
        p2 = galerkin.solve(sp, kk, galerkin.load(sp, np.full_like(kk, grav * rho_w)))
        assert np.allclose(p1, p2, rtol=1e-12, atol=1e-15), (dim, ne, r)
        assert np.max(np.abs(p1)) > 1e-3
        f = galerkin.load(sp, zero, np.full_like(kk, 2.5), grav)
        assert np.max(np.abs(f[galerkin.interior_mask(sp)])) < 1e-14


def test_pressure_solve_matches_direct_assembly():
    ne, r = 8, 2
    sp = Space(ne, r, 2)
    rng = np.random.default_rng(1)
    perm = np.exp(0.5 * rng.standard_normal((ne + 1, ne + 1)))
    q = np.zeros((ne + 1, ne + 1))
    q[3, 3], q[5, 6] = 4.0, -4.0
    s_coefs = rng.uniform(0, 0.5, (sp.nb, sp.nb))
    p = galerkin.pressure_solve(sp, s_coefs, perm, q, 1.0, 0.1, 2.0)
    alpha, _ = galerkin.fields_at_gauss(sp, s_coefs, perm, 1.0, 0.1, 2.0)
    s = galerkin.stiffness(sp, alpha).toarray()
    f = galerkin.load(sp, sp.nodal_at_gauss(q)).ravel()
    m = galerkin.interior_mask(sp).ravel()
    res = (s @ p.ravel() - f)[m]
    assert np.linalg.norm(res) < 1e-12 * np.linalg.norm(f)
    assert np.all(p[~galerkin.interior_mask(sp)] == 0.0)


def test_direct_solver_algorithm_step():
    """One pass of the direct-solver algorithm moves the saturation and
    re-solves the pressure for it; boundary coefficients stay 0."""
    from oracle import Oracle
    from paper_2604_20731_amd import inputs
    p = inputs.make_problem("tiny")
    o = Oracle(p.dim, p.n_elem, p.degree, p.width, p.hidden, p.log_perm, p.porosity,
               np.array([[0.375, 0.5, 1.0], [0.625, 0.5, -1.0]]), p.theta0,
               s0_coefs=np.random.default_rng(2).uniform(0, 0.5, (p.n_elem + p.degree,) * 2))
    p0 = o.galerkin_pressure()
    s0 = o.s.copy()
    p1 = o.step_galerkin(1e-4, p0)
    assert np.max(np.abs(o.s - s0)) > 1e-8
    assert np.max(np.abs(p1 - p0)) > 0
    assert np.all(p1[~galerkin.interior_mask(o.space)] == 0.0)


def test_separable_product_equals_assembled_stiffness():
    rng = np.random.default_rng(7)
    for ne, r in ((6, 1), (7, 2), (5, 3)):
        sp = Space(ne, r, 2)
        ng = len(sp.wg)
        alpha = rng.uniform(0.1, 3.0, ng * ng)
        p = rng.standard_normal((sp.nb, sp.nb))
        s = galerkin.stiffness(sp, alpha)
        sp_p = galerkin.apply_stiffness(sp, alpha, p)
        assert np.abs(sp_p.ravel() - s @ p.ravel()).max() <= 1e-13 * np.abs(s @ p.ravel()).max()
        bound = galerkin.apply_stiffness(sp, alpha, p, absolute=True).ravel()
        exact = abs(s) @ np.abs(p.ravel())
        assert np.all(bound >= exact * (1 - 1e-13))
