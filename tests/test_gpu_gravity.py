"""Gravity on the HIP path against the FP64 oracle (whose gravity terms are
pinned by closed forms and central differences on the CPU): the pressure
right-hand side with the forward-difference divergence of g K sum lambda rho
(eq. 5 on the collocation grid), the gas flux lambda_g K (grad p - rho_g g)
in the explicit saturation update (eq. 9-10), and the log K gradient that the
right-hand side adds.  g points along -y in 2D and -z in 3D.  Saturations
are non-uniform so every gravity term is active."""
import numpy as np
import pytest

from helpers import check, oracle_for, problem, rel, say, scenario_for
from oracle import ads, bspline, cfl_dt

pytestmark = pytest.mark.gpu

GRAV = dict(gravity=2.0, rho_w=1.2, rho_g=0.4)
WELLS3 = np.array([[0.25, 0.25, 1.0], [0.75, 0.75, -1.0]])


def _fp32_tol(ne, r, dim):
    return max(1e-5, np.linalg.cond(bspline.mass_1d(ne, r)) ** dim * 2.0 ** -24)


def _with_s0(prob, seed):
    nb = prob.n_elem + prob.degree
    return np.random.default_rng(seed).uniform(0.0, 0.6, (nb,) * prob.dim)


def _pair(prob, prec, seed=1):
    s0 = _with_s0(prob, seed)
    sc = scenario_for(prob, prec, **GRAV)
    orc = oracle_for(prob, **GRAV)
    sc.set_saturation(s0)
    orc.s = s0.copy()
    orc.refresh()
    return sc, orc, s0


CASES = [("c1", {}), ("c1", dict(n_elem=64, width=64, hidden=4)),
         ("c5", dict(n_elem=8, width=16, hidden=2, wells=WELLS3)),
         ("c5", dict(n_elem=16, width=32, hidden=4, wells=WELLS3))]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3f"])
@pytest.mark.parametrize("name,over", CASES)
def test_loss_and_gradients_with_gravity(prec, name, over):
    say("gravity loss_grad", prec, name, over)
    prob = problem(name, **over)
    if prec == "bf16x3f" and not (prob.width in (32, 64) and prob.hidden in (3, 4)):
        pytest.skip("mixed form: widths 32/64 here, 3-4 hidden layers")
    sc, orc, _ = _pair(prob, prec)
    loss, g, gl = sc.loss_grad(with_logperm=True)
    lref, gref = orc.loss_and_grad()
    glref = orc.loss_grad_logperm()
    el = abs(loss - lref) / abs(lref)
    say(f"  loss {el:.2e}")
    tol = {"fp64": 1e-10, "fp32": 1e-4, "bf16x3f": 1e-4}[prec]
    assert el <= tol
    check("dlogK", gl, glref, tol)
    check("dtheta", g, gref, 3e-3 if prec == "bf16x3f" else tol)
    # the gravity terms matter at this size: without them the loss differs
    orc.gravity = 0.0
    orc.refresh()
    assert abs(orc.loss_and_grad()[0] - lref) > 1e-2 * abs(lref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nsub", [1, 10])
@pytest.mark.parametrize("name,over", [("c1", {}), ("c1", dict(n_elem=40, degree=3)),
                                       ("c5", dict(n_elem=12, width=16, hidden=2, wells=WELLS3))])
def test_saturation_substeps_with_gravity(prec, nsub, name, over):
    say("gravity substeps", prec, nsub, name, over)
    prob = problem(name, **over)
    sc, orc, s0 = _pair(prob, prec, seed=prob.n_elem)
    tau = 0.1 * cfl_dt(orc)
    sc.saturation_substeps(tau, nsub)
    p = ads.project_nodal(orc.space, orc.u_nodal())
    for _ in range(nsub):
        orc.s = ads.saturation_substep(orc.space, orc.s, p, orc.perm, orc.poro, orc.q_inj,
                                       orc.q_prod, tau, orc.mu_w, orc.mu_g, orc.n_exp,
                                       orc.rho_g, orc.gravity)
    orc.refresh()
    _, s_gpu, sn_gpu = sc.fields()
    tol = 1e-12 if prec == "fp64" else _fp32_tol(prob.n_elem, prob.degree, prob.dim) * nsub
    say(f"  S {rel(s_gpu, orc.s):.2e}  dS {rel(s_gpu - s0, orc.s - s0):.2e}")
    check("S", s_gpu, orc.s, tol)
    check("S nodal", sn_gpu, orc.s_nodal, tol)
    check("dS", s_gpu - s0, orc.s - s0, 1e-10 if prec == "fp64" else 1e-3)


# The mixed form (bf16 activations and deltas in the backward) drifts to
# about 6e-3 from the FP64 trajectory over these 500 iterations at C1 size
# with gravity, above the 5e-3 bound of a BF16 network; gravity scenarios
# therefore take the split-bf16 form (three products per weight product in
# the backward too), which is held to 5e-3 here.  The mixed form's
# one-iteration parity with gravity is checked above.
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-3), ("bf16x3", 5e-3)])
def test_coupled_trajectory_with_gravity(prec, tol):
    say("gravity coupled c1", prec)
    prob = problem("c1")
    sc, orc, _ = _pair(prob, prec)
    n_pre = 300
    l_gpu = sc.pretrain_pressure(n_pre)
    orc.pretrain(n_pre)
    assert abs(l_gpu - orc.loss_history[-1]) <= tol * abs(orc.loss_history[-1])
    dt = cfl_dt(orc)
    for k in range(2):
        sc.step(dt)
        orc.step(dt)
        p, s, sn = sc.fields()
        pr, sr, snr = orc.fields()
        say(f"  step {k}: p {rel(p, pr):.3e}  S {rel(s, sr):.3e}  Snodal {rel(sn, snr):.3e}")
        check("p", p, pr, tol)
        check("S", s, sr, tol)
        check("S nodal", sn, snr, tol)
