"""The largest grids the library accepts (2D Ne = 1024 with cubic splines,
3D Ne = 256), where the oracle cannot run the whole path: the Kronecker mass
solve (eq. 14) and the Gram solve (eq. 26-28) checked by properties that hold
at any size.  The GPU solution is put back through the operator, applied on
the CPU from its definition (the 1D B-spline mass matrices along every axis;
the integer 5-point stencil in 2D, h times the 7-point stencil in 3D, zero
outside the interior).  The criterion is the normwise backward error
|A x - b| / (|A|_2 |x|), which a stable solve keeps at a small multiple of
the unit round-off whatever the size and conditioning (the Gram matrix at
Ne = 1024 has condition number ~1e6, so a residual relative to |b| alone is
no size-independent measure): bound 64 u, u = 2^-24 (float32) or 2^-53."""
import numpy as np
import pytest

from helpers import problem, say, scenario_for
from oracle import bspline
from oracle.ads import along

pytestmark = pytest.mark.gpu

WELLS3 = np.array([[0.25, 0.25, 1.0], [0.75, 0.75, -1.0]])


def _apply_mass(x, ne, r):
    m1 = bspline.mass_1d(ne, r)
    out = x
    for ax in range(x.ndim):
        out = along(m1, out, ax)
    return out


def _apply_gram(q):
    dim = q.ndim
    pad = np.pad(q, 1)
    core = tuple(slice(1, -1) for _ in range(dim))
    out = 2.0 * dim * q
    for ax in range(dim):
        for sh in (-1, 1):
            sl = list(core)
            sl[ax] = slice(1 + sh, pad.shape[ax] - 1 + sh)
            out = out - pad[tuple(sl)]
    if dim == 3:
        out = out / (q.shape[0] + 1)   # h = 1/Ne, interior width Ne - 1
    return out


def _prob(dim):
    if dim == 2:
        return problem("c1", n_elem=1024, degree=3, width=16, hidden=2)
    return problem("c5", n_elem=256, degree=2, width=16, hidden=2, wells=WELLS3)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dim,prec", [(2, "fp64"), (2, "fp32"), (3, "fp32")])
def test_mass_and_gram_solves_at_maximum_size(dim, prec):
    prob = _prob(dim)
    say("max size", dim, prec, prob.n_elem, prob.degree)
    sc = scenario_for(prob, prec)
    rng = np.random.default_rng(dim)
    nb = prob.n_elem + prob.degree
    b = rng.standard_normal((nb,) * dim)
    u = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
    x = sc.mass_solve(b).reshape(b.shape)
    norm_m = np.linalg.norm(bspline.mass_1d(prob.n_elem, prob.degree), 2) ** dim
    e_m = np.linalg.norm(_apply_mass(x, prob.n_elem, prob.degree) - b) / (norm_m * np.linalg.norm(x))
    m = prob.n_elem - 1
    res = rng.standard_normal((m,) * dim)
    q = sc.gram_solve(res).reshape(res.shape)
    norm_g = 4.0 * dim * (1.0 / prob.n_elem if dim == 3 else 1.0)
    e_g = np.linalg.norm(_apply_gram(q) - res) / (norm_g * np.linalg.norm(q))
    say(f"  backward error: mass {e_m / u:.1f} u, gram {e_g / u:.1f} u")
    assert e_m < 64 * u and e_g < 64 * u
    sc.close()
