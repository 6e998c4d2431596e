"""Parity of the 3D path (d = 3: seven-point residual, Gram G = h L7 solved by
DST-I along z and y with shifted line solves along x, trilinear projection,
sum-factorised saturation assembly, three-direction Kronecker mass solve,
3-input network) with the FP64 oracle on identical seeded inputs."""
import numpy as np
import pytest

from helpers import check, oracle_for, problem, rel, say, scenario_for
from oracle import ads, bspline, cfl_dt, pressure

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 1e-5}
# two vertical wells on node columns of every grid used here
WELLS = np.array([[0.25, 0.25, 1.0], [0.75, 0.75, -1.0]])


def fp32_tol(ne, r):
    """FP32 bound for results that pass through M^-1: rounding of the
    right-hand side (relative 2^-24) amplified by at most cond(M) =
    cond(M_1)^3, never below the 1e-5 ADS criterion.  Cubic 3D: about 1e-3,
    quadratic about 7e-5, linear 1e-5."""
    return max(1e-5, np.linalg.cond(bspline.mass_1d(ne, r)) ** 3 * 2.0 ** -24)


def prob3(ne, r=2, width=32, hidden=4, **kw):
    return problem("c5", n_elem=ne, degree=r, width=width, hidden=hidden, wells=WELLS, **kw)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ne,r", [(12, 2), (8, 3), (20, 2), (37, 1)])
def test_mass_solve_3d(prec, ne, r):
    say("mass_solve_3d", prec, ne, r)
    sc = scenario_for(prob3(ne, r, width=16, hidden=2), prec)
    sp_ = ads.Space(ne, r, 3)
    b = np.random.default_rng(ne + r).standard_normal((sp_.nb,) * 3)
    check("x", sc.mass_solve(b), sp_.mass_solve(b), TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ne", [8, 20, 65, 70])
def test_gram_solve_3d(prec, ne):
    """m = 64 fills the padded pitch exactly; m = 69 leaves 59 padded modes
    per axis, whose lines must stay zero."""
    say("gram_solve_3d", prec, ne)
    sc = scenario_for(prob3(ne, width=16, hidden=2), prec)
    res = np.random.default_rng(ne).standard_normal((ne - 1,) * 3)
    q = sc.gram_solve(res)
    check("q", q, pressure.gram_solve(res), TOL[prec] * 10)


@pytest.mark.parametrize("prec,ne,width,hidden", [
    ("fp64", 8, 16, 2), ("fp64", 12, 32, 4), ("fp32", 12, 16, 2), ("fp32", 12, 32, 4),
    ("fp32", 17, 64, 4), ("bf16x3", 12, 32, 4), ("bf16x3", 17, 64, 4), ("bf16", 12, 128, 4),
    ("bf16x3f", 12, 128, 4)])
def test_loss_and_gradients_3d(prec, ne, width, hidden):
    """Widths 32/64/128 with 4 hidden layers take the matrix-core network in
    fp32/bf16x3/bf16; 13^3 and 18^3 nodes leave a partial last tile."""
    say("loss_grad_3d", prec, ne, width, hidden)
    prob = prob3(ne, width=width, hidden=hidden)
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob)
    loss, g, gl = sc.loss_grad(with_logperm=True)
    lref, gref = orc.loss_and_grad()
    glref = orc.loss_grad_logperm()
    el = abs(loss - lref) / abs(lref)
    say(f"  loss {el:.2e}")
    tol = {"fp64": 1e-10, "fp32": 1e-4, "bf16": 1e-1, "bf16x3": 1e-4, "bf16x3f": 1e-4}[prec]
    # mixed form: bf16 activations and deltas in the backward (dtheta 3e-3)
    assert el <= tol
    check("dlogK", gl, glref, tol)
    check("dtheta", g, gref, 3e-3 if prec == "bf16x3f" else tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ne,r", [(8, 2), (12, 3), (20, 1)])
def test_projection_3d(prec, ne, r):
    say("projection_3d", prec, ne, r)
    prob = prob3(ne, r, width=16, hidden=2)
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob)
    pref = ads.project_nodal(orc.space, orc.u_nodal())
    check("p", sc.project_pressure(), pref, 1e-11 if prec == "fp64" else fp32_tol(ne, r))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nsub", [1, 10])
@pytest.mark.parametrize("ne,r", [(8, 2), (12, 3), (16, 1), (20, 2)])
def test_saturation_substeps_3d(prec, nsub, ne, r):
    say("substeps_3d", prec, nsub, ne, r)
    prob = prob3(ne, r, width=16, hidden=2)
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob)
    nb = ne + r
    s0 = np.random.default_rng(ne).uniform(0.0, 0.6, (nb,) * 3)
    sc.set_saturation(s0)
    orc.s = s0.copy()
    orc.refresh()
    tau = 0.1 * cfl_dt(orc)
    sc.saturation_substeps(tau, nsub)
    p = ads.project_nodal(orc.space, orc.u_nodal())
    for _ in range(nsub):
        orc.s = ads.saturation_substep(orc.space, orc.s, p, orc.perm, orc.poro, orc.q_inj,
                                       orc.q_prod, tau, orc.mu_w, orc.mu_g, orc.n_exp)
    orc.refresh()
    _, s_gpu, sn_gpu = sc.fields()
    tol = 1e-12 if prec == "fp64" else fp32_tol(ne, r) * nsub
    check("S", s_gpu, orc.s, tol)
    check("S nodal", sn_gpu, orc.s_nodal, tol)
    check("dS", s_gpu - s0, orc.s - s0, 1e-10 if prec == "fp64" else 1e-3)


@pytest.mark.parametrize("prec,width,tol", [("fp64", 16, 1e-8), ("fp32", 32, 1e-3),
                                            ("bf16x3", 32, 5e-3)])
def test_coupled_trajectory_3d(prec, width, tol):
    """13^3 nodes, two vertical wells: pretraining, then coupled steps."""
    say("coupled_3d", prec, width)
    prob = prob3(12, width=width, hidden=4 if width == 32 else 2)
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob, lr=1e-4)
    n_pre, n_steps = 200, 2
    l_gpu = sc.pretrain_pressure(n_pre)
    orc.pretrain(n_pre)
    assert abs(l_gpu - orc.loss_history[-1]) <= tol * abs(orc.loss_history[-1])
    dt = cfl_dt(orc)
    for k in range(n_steps):
        sc.step(dt)
        orc.step(dt)
        p, s, sn = sc.fields()
        pr, sr, snr = orc.fields()
        say(f"  step {k}: p {rel(p, pr):.3e}  S {rel(s, sr):.3e}  Snodal {rel(sn, snr):.3e}")
        check("p", p, pr, tol)
        check("S", s, sr, tol)
        check("S nodal", sn, snr, tol)


@pytest.mark.timeout(600)
def test_coupled_trajectory_3d_c5_network():
    """The C5 network (3 -> 4x128 -> 1) in the mixed form, the serving and
    precision default, on a 25^3-node grid with two vertical wells: 200
    pretraining iterations and two coupled steps against the FP64 oracle at
    the BF16-network tolerance 5e-3."""
    say("coupled_3d c5 network, bf16x3f")
    tol = 5e-3
    prob = prob3(24, width=128, hidden=4)
    sc = scenario_for(prob, "bf16x3f")
    orc = oracle_for(prob, lr=1e-4)
    n_pre = 200
    l_gpu = sc.pretrain_pressure(n_pre)
    orc.pretrain(n_pre)
    assert abs(l_gpu - orc.loss_history[-1]) <= tol * abs(orc.loss_history[-1])
    dt = cfl_dt(orc)
    for k in range(2):
        sc.step(dt)
        orc.step(dt)
        p, s, sn = sc.fields()
        pr, sr, snr = orc.fields()
        say(f"  step {k}")
        check("p", p, pr, tol)
        check("S", s, sr, tol)
        check("S nodal", sn, snr, tol)
