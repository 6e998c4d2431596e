"""The distance form of the trial-function factor (u = prod 4 x (1 - x) NN)
against the oracle, through both network kernel families (per-node float64,
matrix-core float32 and split bf16, 2D and 3D): the network pressure, the
loss and dLOSS/dtheta at moved parameters, and a short coupled trajectory.
Also the library's seeded default parameters (crv_init with theta0 NULL)
against SplitMix64 and the Xavier rule as the tests' helpers write them out."""
import numpy as np
import pytest

from helpers import (check, default_theta, maxrel, oracle_for, problem, rel, say,
                     scenario_for)
from oracle import cfl_dt

pytestmark = pytest.mark.gpu

WELLS3 = np.array([[0.25, 0.25, 1.0], [0.75, 0.75, -1.0]])


@pytest.mark.parametrize("name,prec,over,tol,tol_g", [
    ("c1", "fp64", {}, 1e-10, 1e-10),
    ("c1", "fp32", {}, 3e-5, 1e-4),
    ("c2", "bf16x3f", {}, 1e-4, 3e-3),
    ("c5", "fp32", dict(n_elem=16, width=32, hidden=4, wells=WELLS3), 3e-5, 1e-4),
])
def test_distance_factor_loss_grad(name, prec, over, tol, tol_g):
    """tol bounds the network pressure (relative L2 and max error over max |p|):
    float32 products and tanh through the layers give about 1e-5 at the
    largest node (measured 5e-6 L2, 1.0e-5 max at 33^2); tol_g bounds the loss
    and dtheta (the mixed form's bf16 backward: 3e-3)."""
    say("distance factor loss/grad", name, prec)
    prob = problem(name, **over)
    sc = scenario_for(prob, prec, boundary_factor=1)
    orc = oracle_for(prob, boundary_factor=1)
    th = prob.theta0 + 0.05 * np.random.default_rng(3).standard_normal(prob.theta0.size)
    sc.set_theta(th)
    loss, g = sc.loss_grad()
    lref, gref = orc.loss_and_grad(th)
    p = sc.fields()[0]
    pref = orc.u_nodal(th)
    e = dict(p=rel(p, pref), p_max=np.max(np.abs(p - pref)) / np.max(np.abs(pref)),
             loss=abs(loss - lref) / abs(lref), dtheta=rel(g, gref), dtheta_max=maxrel(g, gref))
    say("  " + "  ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert e["p"] < tol and e["p_max"] < tol and e["loss"] < tol_g, e
    assert e["dtheta"] < tol_g and e["dtheta_max"] < tol_g, e
    # the factor vanishes on the boundary and the indicator form differs inside
    assert np.all(p[0] == 0) and np.all(p[-1] == 0) and np.all(p[..., 0] == 0)
    sc.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-3), ("bf16x3f", 5e-3)])
def test_distance_factor_trajectory_c1(prec, tol):
    say("distance factor trajectory c1", prec)
    prob = problem("c1")
    sc = scenario_for(prob, prec, boundary_factor=1)
    orc = oracle_for(prob, lr=1e-4, boundary_factor=1)
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
        say(f"  step {k}: p {rel(p, pr):.3e}  S {rel(s, sr):.3e}")
        check("p", p, pr, tol)
        check("S", s, sr, tol)
        check("S nodal", sn, snr, tol)
    sc.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_seeded_default_theta(prec):
    """crv_init with theta0 NULL: Xavier-uniform weights from SplitMix64 in
    layout order, zero biases; float32 contexts hold them rounded once."""
    from paper_2604_20731_amd import crv
    say("seeded default theta", prec)
    prob = problem("c1")
    cfg = crv.config(dim=2, n_elem=prob.n_elem, degree=prob.degree, width=prob.width,
                     hidden=prob.hidden, precision=prec)
    ref = {s: default_theta(2, prob.width, prob.hidden, s) for s in (0, 99)}
    for seed in (0, 99):
        sc = crv.Scenario(cfg, prob.log_perm, prob.porosity, prob.wells, None, seed=seed)
        th = sc.get_state()[0]
        want = ref[seed] if prec == "fp64" else ref[seed].astype(np.float32).astype(np.float64)
        assert np.array_equal(th, want)
        sc.close()
    assert not np.array_equal(ref[0], ref[99])
