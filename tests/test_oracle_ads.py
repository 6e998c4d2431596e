"""Pins of the oracle's IGA-ADS pieces: Kronecker mass solve against the
literal dense Kronecker system and LAPACK banded Cholesky, projection
reproducing bilinear data, conservation and source balance of the explicit
substep, and the flux term against the analytic divergence."""
import numpy as np
import pytest

from oracle import ads, bspline, wells


@pytest.mark.parametrize("dim,ne,r", [(2, 32, 2), (2, 9, 3), (3, 6, 2)])
def test_mass_solve_variants_agree(dim, ne, r):
    sp_ = ads.Space(ne, r, dim)
    b = np.random.default_rng(0).standard_normal((sp_.nb,) * dim)
    x_dense = sp_.mass_solve_dense_kron(b)
    assert np.allclose(sp_.mass_solve(b), x_dense, rtol=1e-10, atol=1e-10)
    assert np.allclose(sp_.mass_solve_banded(b), x_dense, rtol=1e-10, atol=1e-10)
    # residual of the literal system
    assert np.allclose(sp_.mass_full() @ x_dense.ravel(), b.ravel(), atol=1e-12)


@pytest.mark.parametrize("dim,r", [(2, 2), (2, 3), (3, 2)])
def test_projection_reproduces_multilinear_data(dim, r):
    ne = 7
    sp_ = ads.Space(ne, r, dim)
    x = bspline.node_points(ne)
    grids = np.meshgrid(*([x] * dim), indexing="ij")[::-1]     # x, y[, z]
    coeffs = [0.3, -1.2, 0.7, 2.0]
    u = coeffs[0] + coeffs[1] * grids[0] + coeffs[2] * grids[1] + coeffs[3] * grids[0] * grids[1]
    if dim == 3:
        u = u + 0.4 * grids[2] * grids[0]
    u = np.transpose(u) if dim == 2 else np.transpose(u, (2, 1, 0))
    p = ads.project_nodal(sp_, u)
    g = sp_.xg
    gg = np.meshgrid(*([g] * dim), indexing="ij")[::-1]
    ref = coeffs[0] + coeffs[1] * gg[0] + coeffs[2] * gg[1] + coeffs[3] * gg[0] * gg[1]
    if dim == 3:
        ref = ref + 0.4 * gg[2] * gg[0]
    ref = np.transpose(ref) if dim == 2 else np.transpose(ref, (2, 1, 0))
    assert np.allclose(sp_.at_gauss(p), ref, atol=1e-12)
    # nodal values are reproduced too
    assert np.allclose(sp_.at_nodes(p), u, atol=1e-12)


def _integral(sp_, c):
    return float(np.sum(sp_.mass_full() @ c.ravel()))


@pytest.mark.parametrize("dim", [2, 3])
def test_substep_conserves_mass_without_sources(dim):
    ne = 8 if dim == 2 else 5
    rng = np.random.default_rng(1)
    sp_ = ads.Space(ne, 2, dim)
    s = rng.uniform(0, 1, (sp_.nb,) * dim)
    p = rng.standard_normal((sp_.nb,) * dim)
    perm = np.exp(rng.standard_normal((ne + 1,) * dim))
    poro = rng.uniform(0.1, 0.3, (ne + 1,) * dim)
    z = np.zeros((ne + 1,) * dim)
    s1 = ads.saturation_substep(sp_, s, p, perm, poro, z, z, 1e-3, 1.0, 0.1, 2.0)
    assert abs(_integral(sp_, s1) - _integral(sp_, s)) < 1e-13
    assert np.max(np.abs(s1 - s)) > 1e-6            # the flux did move saturation
    # no pressure gradient and no source: nothing changes
    s2 = ads.saturation_substep(sp_, s, np.ones_like(p), perm, poro, z, z, 1e-3, 1.0, 0.1, 2.0)
    assert np.allclose(s2, s, atol=1e-12)


def test_substep_source_balance():
    ne = 24
    sp_ = ads.Space(ne, 2, 2)
    w = np.array([[0.3, 0.4, 1.0], [0.7, 0.6, -0.5]])
    qi, qp = wells.nodal_sources(w, ne, 2, 0.06)
    poro = np.full((ne + 1, ne + 1), 0.2)
    perm = np.ones_like(poro)
    tau = 1e-3
    # S = 0.5 everywhere (partition of unity), p constant: f_g(0.5) = 10/11
    s = np.full((sp_.nb, sp_.nb), 0.5)
    s1 = ads.saturation_substep(sp_, s, np.zeros_like(s), perm, poro, qi, qp, tau, 1.0, 0.1, 2.0)
    gain = _integral(sp_, s1) - _integral(sp_, s)
    assert abs(gain - tau / 0.2 * (1.0 + 10.0 / 11.0 * -0.5)) < 1e-13
    # S = 0: producers remove no gas
    s0 = np.zeros_like(s)
    s1 = ads.saturation_substep(sp_, s0, np.zeros_like(s), perm, poro, qi, qp, tau, 1.0, 0.1, 2.0)
    assert abs(_integral(sp_, s1) - tau / 0.2 * 1.0) < 1e-13


def _greville(ne, r):
    t = bspline.knot_vector(ne, r)
    return np.array([t[i + 1:i + r + 1].mean() for i in range(ne + r)])


@pytest.mark.parametrize("ne", [32, 64])
def test_flux_term_matches_analytic_divergence(ne):
    """(b - M S)/tau is the projection of phi^-1 div(lambda_g(S) K grad p) for a
    saturation bump away from the boundary; p = -x, K = 1."""
    r, phi, mu_g = 2, 0.2, 0.1
    sp_ = ads.Space(ne, r, 2)
    x = bspline.node_points(ne)
    xx, yy = np.meshgrid(x, x, indexing="xy")
    bump = 0.8 * np.exp(-((xx - 0.5) ** 2 + (yy - 0.5) ** 2) / (2 * 0.08 ** 2))
    s = ads.project_nodal(sp_, bump)
    p = np.tile(-_greville(ne, r)[None, :], (sp_.nb, 1))            # p = -x exactly
    assert np.allclose(sp_.at_gauss(p, deriv_axis=0), -1.0)
    z = np.zeros((ne + 1, ne + 1))
    tau = 1.0
    b = ads.saturation_rhs(sp_, s, p, np.ones_like(z), np.full_like(z, phi), z, z, tau, 1.0, mu_g, 2.0)
    flux = sp_.mass_solve(b - (sp_.mass_full() @ s.ravel()).reshape(s.shape)) / tau
    sg = sp_.at_gauss(s)
    dsx = sp_.at_gauss(s, deriv_axis=0)
    # div(lambda_g(S) K grad p)/phi with grad p = (-1, 0), lambda_g = s^2/mu_g (s in [0,1])
    sc = np.clip(sg, 0, 1)
    ref = -(2.0 * sc * (sg > 0) * (sg < 1) / mu_g) * dsx / phi
    err = np.sqrt(np.sum((sp_.at_gauss(flux) - ref) ** 2) / np.sum(ref ** 2))
    assert err < (0.05 if ne == 32 else 0.015)


def test_wells_nodal_sources_balance_and_errors():
    ne = 40
    w = np.array([[0.3, 0.4, 1.0], [0.7, 0.6, -0.5], [0.5, 0.5, 0.25]])
    qi, qp = wells.nodal_sources(w, ne, 2, 0.06)
    h = 1.0 / ne
    assert abs(h * h * qi.sum() - 1.25) < 1e-13 and abs(h * h * qp.sum() + 0.5) < 1e-13
    qi3, qp3 = wells.nodal_sources(w[:1], 10, 3, 0.12)
    assert abs(qi3.sum() / 1000.0 - 1.0) < 1e-13 and qp3.sum() == 0
    with pytest.raises(ValueError):
        wells.nodal_sources(np.array([[0.02, 0.5, 1.0]]), ne, 2, 0.06)
    with pytest.raises(ValueError):
        wells.nodal_sources(np.array([[0.4, 0.4, 1.0]]), 4, 2, 0.06)
