"""The paper's direct-solver pressure path on the HIP side (matrix-free
Galerkin operator, CG preconditioned by the diagonal of S or by the scaled
Kronecker inverse; 2D) against the oracle's
sparse direct solve of the same system (eq. 15-20; pinned on the CPU by an
exactly reproduced polynomial pressure and the gravity load identity)."""
import numpy as np
import pytest

from helpers import check, oracle_for, problem, rel, say, scenario_for
from oracle import cfl_dt

pytestmark = pytest.mark.gpu

GRAV = dict(gravity=2.0, rho_w=1.2, rho_g=0.4)


def _pair(prob, prec, grav, seed=3):
    nb = prob.n_elem + prob.degree
    s0 = np.random.default_rng(seed).uniform(0.0, 0.6, (nb, nb))
    kw = GRAV if grav else {}
    sc = scenario_for(prob, prec, **kw)
    orc = oracle_for(prob, **kw)
    sc.set_saturation(s0)
    orc.s = s0.copy()
    orc.refresh()
    return sc, orc


# CG to rtol 1e-12 (FP64) agrees with the direct solve to about the
# preconditioned condition number times rtol; FP32 to rtol 1e-6 lands within
# that condition number (~10-100 here) times 2^-24 and rtol (measured <= 8e-7)
@pytest.mark.parametrize("prec,rtol,tol", [("fp64", 1e-12, 1e-8), ("fp32", 1e-6, 1e-5)])
@pytest.mark.parametrize("ne,r", [(32, 2), (24, 3), (40, 1), (64, 2)])
@pytest.mark.parametrize("grav", [False, True])
@pytest.mark.parametrize("precond", ["jacobi", "kron"])
def test_galerkin_pressure_matches_direct_solve(prec, rtol, tol, ne, r, grav, precond):
    say("galerkin", prec, ne, r, grav, precond)
    prob = problem("c1", n_elem=ne, degree=r)
    sc, orc = _pair(prob, prec, grav)
    p, iters, rr = sc.pressure_galerkin(max_iters=20000, rtol=rtol, precond=precond)
    pref = orc.galerkin_pressure()
    say(f"  iters {iters} |r|/|F| {rr:.2e}")
    assert rr <= rtol * 1.0001 or prec == "fp32"
    check("P", p, pref.ravel(), tol)


# FP32: each substep passes through M^-1 (bound 1e-5 per substep, as for the
# collocation path's substeps), ten per pass
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-4)])
def test_direct_solver_algorithm_steps(prec, tol):
    """Two passes of the direct-solver algorithm (substeps with the Galerkin
    pressure, refresh, new Galerkin pressure) against the oracle."""
    say("galerkin steps", prec)
    prob = problem("c1")
    sc, orc = _pair(prob, prec, grav=True)
    rtol = 1e-12 if prec == "fp64" else 1e-6
    sc.pressure_galerkin(rtol=rtol)
    p = orc.galerkin_pressure()
    dt = cfl_dt(orc)
    for k in range(2):
        sc.step_galerkin(dt, rtol=rtol)
        p = orc.step_galerkin(dt, p)
        _, s_gpu, _ = sc.fields()
        check(f"step {k} S", s_gpu, orc.s, tol)
    p_gpu, _, _ = sc.pressure_galerkin(rtol=rtol)
    check("P", p_gpu, p.ravel(), tol)


def test_galerkin_path_rejects_3d():
    from paper_2604_20731_amd import crv
    prob = problem("c5", n_elem=8, width=16, hidden=2, wells=np.array([[0.5, 0.5, 1.0]]))
    sc = scenario_for(prob, "fp32")
    with pytest.raises(crv.CrvError, match="2D"):
        sc.pressure_galerkin()


@pytest.mark.parametrize("precond,min_iters", [("jacobi", 48), ("kron", 25)])
def test_captured_cg_chunks_equal_eager_launches(precond, min_iters):
    """The CG iterations replayed from a captured graph (chunks of 24, the
    host reading the residual between replays, the iterations stopping
    themselves on the device inside a chunk) give bitwise the result and the
    iteration count of the same iterations launched one by one; rtol 1e-9
    takes both preconditioners past the first chunk."""
    import os
    prob = problem("c1", n_elem=48)
    sc_graph, _ = _pair(prob, "fp32", grav=True)
    os.environ["CRV_NO_GRAPH"] = "1"
    try:
        sc_eager, _ = _pair(prob, "fp32", grav=True)
    finally:
        del os.environ["CRV_NO_GRAPH"]
    for _ in range(2):  # the second solve replays the graph captured by the first
        pg, ig, rg = sc_graph.pressure_galerkin(rtol=1e-9, precond=precond)
        pe, ie, re = sc_eager.pressure_galerkin(rtol=1e-9, precond=precond)
        assert ig == ie and rg == re and np.array_equal(pg, pe)
        assert ig >= min_iters


@pytest.mark.timeout(600)
def test_galerkin_at_the_benchmark_size():
    """The 512^2 workload the benchmark times (514^2 coefficients, FP32, rtol
    1e-6) against the oracle's sparse LU of the same system, with both
    preconditioners: the same bound as at the small sizes, 1e-5 (measured
    8.4e-7 with the diagonal).  The Kronecker inverse's iteration count does
    not grow with the mesh as the diagonal's does: well under half of it
    here."""
    say("galerkin 512^2")
    prob = problem("b512")
    sc = scenario_for(prob, "fp32")
    orc = oracle_for(prob)
    pref = orc.galerkin_pressure().ravel()
    its = {}
    for precond in ("jacobi", "kron"):
        p, its[precond], rr = sc.pressure_galerkin(rtol=1e-6, precond=precond)
        say(f"  {precond}: iters {its[precond]} |r|/|F| {rr:.2e}")
        assert rr <= 1e-6
        check(f"{precond} P", p, pref, 1e-5)
    assert its["kron"] < 0.5 * its["jacobi"]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precond", ["kron", "jacobi"])
def test_galerkin_at_the_largest_mesh(precond):
    """1024^2 cubic elements, the largest 2D mesh (1027^2 coefficients; the
    Kronecker work arrays padded from 1025 to 1088 per axis, 8 x 8 operator
    tiles): no direct solve fits here, so the FP32 solution is judged by its
    true residual, evaluated in FP64 by the oracle axis by axis.  A CG
    solution stored in FP32 has a residual of order u |S| |P| from its own
    rounding (|S| |P| is about cond(S) |F|, so |F - S P| / |F| alone is not
    a size-independent criterion), plus the gap between the recursively
    updated and the true residual: |F - S P| <= 2 rtol |F| + 64 u || |S| |P| ||
    (the normwise backward-error bound of the other maximum-size solves;
    measured 1.1 u with the Kronecker preconditioner in 255 iterations,
    2.5 u with the diagonal in 1334)."""
    from oracle import galerkin
    say("galerkin 1024^2 cubic", precond)
    prob = problem("c3", width=64)
    sc = scenario_for(prob, "fp32")
    orc = oracle_for(prob)
    rtol = 1e-6
    p, iters, rr = sc.pressure_galerkin(max_iters=20000, rtol=rtol, precond=precond)
    spc = orc.space
    alpha, flux = galerkin.fields_at_gauss(spc, orc.s, orc.perm, orc.mu_w, orc.mu_g, orc.n_exp,
                                           orc.rho_w, orc.rho_g)
    f = galerkin.load(spc, spc.nodal_at_gauss(orc.q), flux, orc.gravity)
    inner = galerkin.interior_mask(spc)
    P = p.reshape(spc.nb, spc.nb)
    assert np.all(P[~inner] == 0)
    res = (f - galerkin.apply_stiffness(spc, alpha, P))[inner]
    size = galerkin.apply_stiffness(spc, alpha, P, absolute=True)[inner]
    fn, rn, sn = np.linalg.norm(f[inner]), np.linalg.norm(res), np.linalg.norm(size)
    u = 2.0 ** -24
    say(f"  iters {iters} recursive |r|/|F| {rr:.2e}  true |r|/|F| {rn / fn:.2e}  "
        f"|r| / (u || |S||P| ||) {rn / (u * sn):.1f}")
    assert rr <= rtol
    assert rn <= 2 * rtol * fn + 64 * u * sn


def test_galerkin_rejects_an_unknown_preconditioner():
    """precond outside CRV_PRECOND_* is CRV_EINVAL before any device work;
    the context stays usable."""
    import ctypes as C
    from paper_2604_20731_amd import crv
    prob = problem("c1")
    sc = scenario_for(prob, "fp32")
    it, rr = C.c_int(), C.c_double()
    for bad in (-1, 2, 7):
        assert crv.LIB.crv_pressure_galerkin(sc.ctx, 10, 1e-6, bad, None, C.byref(it),
                                             C.byref(rr)) == crv.CRV_EINVAL
        assert "precond" in crv.LIB.crv_last_error().decode()
        assert crv.LIB.crv_step_galerkin(sc.ctx, 1e-4, 10, 1e-6, bad, None, None) == crv.CRV_EINVAL
    with pytest.raises(KeyError):
        sc.pressure_galerkin(precond="multigrid")
    _, iters, rr = sc.pressure_galerkin(rtol=1e-6)
    assert rr <= 1e-6 and iters > 0


def test_iteration_count_is_exact():
    """The solve stops after the first iteration whose residual meets rtol
    (tested on the device after every iteration, not per chunk of 24): with
    max_iters one less than that count the residual is still above rtol, and
    a solve limited to max_iters iterations does exactly max_iters."""
    prob = problem("c1", n_elem=48)
    for precond in ("jacobi", "kron"):
        sc, _ = _pair(prob, "fp32", grav=True)
        _, n, rr = sc.pressure_galerkin(rtol=1e-6, precond=precond)
        assert rr <= 1e-6 and n > 5
        _, n1, rr1 = sc.pressure_galerkin(max_iters=n - 1, rtol=1e-6, precond=precond)
        assert n1 == n - 1 and rr1 > 1e-6
        _, n2, _ = sc.pressure_galerkin(max_iters=5, rtol=1e-6, precond=precond)
        assert n2 == 5
        say(f"  {precond}: {n} iterations")
