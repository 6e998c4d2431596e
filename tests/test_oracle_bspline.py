"""Pins of the oracle's B-spline space (closed forms, library comparator)."""
import numpy as np
import pytest
import scipy.interpolate

from oracle import bspline


@pytest.mark.parametrize("r", [1, 2, 3])
@pytest.mark.parametrize("ne", [1, 3, 8])
def test_partition_of_unity(r, ne):
    x = np.linspace(0.0, 1.0, 101)
    b = bspline.basis(ne, r, x)
    assert b.shape == (101, ne + r)
    assert np.max(np.abs(b.sum(axis=1) - 1.0)) < 1e-14
    assert np.all(b >= -1e-15)


@pytest.mark.parametrize("r", [2, 3])
@pytest.mark.parametrize("deriv", [0, 1])
def test_against_scipy_bspline(r, deriv):
    ne = 7
    t = bspline.knot_vector(ne, r)
    x = np.linspace(0.0, 1.0, 57)[:-1] + 0.003   # inside [0,1)
    mine = bspline.basis(ne, r, x, deriv=deriv)
    for i in range(ne + r):
        c = np.zeros(ne + r)
        c[i] = 1.0
        spl = scipy.interpolate.BSpline(t, c, r, extrapolate=False)
        ref = spl(x, nu=deriv)
        assert np.allclose(mine[:, i], ref, atol=1e-12), i


def test_knot_values_closed_form():
    # quadratic: (1/2, 1/2) at interior knots; cubic: (1/6, 2/3, 1/6) away from the ends
    ne = 10
    b2 = bspline.basis(ne, 2, bspline.node_points(ne))
    for i in range(1, ne):
        assert np.allclose(b2[i, i:i + 2], [0.5, 0.5])
        assert abs(b2[i].sum() - 1.0) < 1e-15
    b3 = bspline.basis(ne, 3, bspline.node_points(ne))
    for i in range(2, ne - 1):
        assert np.allclose(b3[i, i:i + 3], [1 / 6, 2 / 3, 1 / 6])
    assert b2[0, 0] == 1.0 and b2[-1, -1] == 1.0


def test_mass_interior_rows_closed_form():
    ne = 12
    h = 1.0 / ne
    m2 = bspline.mass_1d(ne, 2)
    row = m2[6, 4:9]
    assert np.allclose(row, h / 120.0 * np.array([1, 26, 66, 26, 1]), atol=1e-15)
    m3 = bspline.mass_1d(ne, 3)
    row = m3[7, 4:11]
    assert np.allclose(row, h / 5040.0 * np.array([1, 120, 1191, 2416, 1191, 120, 1]), atol=1e-15)
    # bandwidth r, symmetric
    assert np.allclose(m2, m2.T) and np.allclose(np.triu(m2, 3), 0)


@pytest.mark.parametrize("r", [2, 3])
def test_mass_row_sums_are_basis_integrals(r):
    ne = 9
    t = bspline.knot_vector(ne, r)
    m = bspline.mass_1d(ne, r)
    integ = (t[r + 1:] - t[:-(r + 1)]) / (r + 1)   # int B_i = (t_{i+r+1}-t_i)/(r+1)
    assert np.allclose(m.sum(axis=1), integ, atol=1e-15)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_gauss_rule_exact_to_degree_2r_plus_1(r):
    xg, wg = bspline.gauss_rule(5, r)
    for k in range(2 * r + 2):
        assert abs(np.sum(wg * xg ** k) - 1.0 / (k + 1)) < 1e-14


def test_hat_interpolates_linear_functions():
    ne = 6
    x = np.linspace(0, 1, 31)
    hm = bspline.hat(ne, x)
    nodes = bspline.node_points(ne)
    assert np.allclose(hm @ (3.0 - 2.0 * nodes), 3.0 - 2.0 * x)
    assert np.allclose(hm.sum(axis=1), 1.0)
