"""Parity of the HIP path (through the C ABI) with the FP64 oracle, piece by
piece on identical seeded inputs: Kronecker mass solve (ADS, tolerance 1e-5
relative in FP32), Gram solve, robust loss and its gradients, pressure
projection, saturation substeps, and short coupled trajectories.  FP64 runs
of the same kernels must agree to round-off."""
import numpy as np
import pytest

from helpers import check, oracle_for, problem, rel, say, scenario_for
from oracle import ads, cfl_dt, pressure

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 1e-5}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ne,r", [(8, 2), (32, 2), (48, 3), (256, 2), (63, 1)])
def test_mass_solve(prec, ne, r):
    say("mass_solve", prec, ne, r)
    prob = problem("c1", n_elem=ne, degree=r)
    sc = scenario_for(prob, prec)
    sp_ = ads.Space(ne, r, 2)
    b = np.random.default_rng(ne + r).standard_normal((sp_.nb, sp_.nb))
    x = sc.mass_solve(b)
    check("x", x, sp_.mass_solve(b), TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ne", [8, 32, 65, 256, 512])
def test_gram_solve(prec, ne):
    say("gram_solve", prec, ne)
    prob = problem("c1", n_elem=ne)
    sc = scenario_for(prob, prec)
    res = np.random.default_rng(ne).standard_normal((ne - 1, ne - 1))
    q = sc.gram_solve(res)
    check("q", q, pressure.gram_solve(res), TOL[prec] * (10 if ne >= 256 else 1))


GRAD_CASES = [("tiny", {}), ("c1", {}), ("c1", dict(n_elem=40, width=64, hidden=4)),
              ("c1", dict(degree=3, width=16, hidden=2)), ("c1", dict(n_elem=256, width=64, hidden=4)),
              ("c1", dict(n_elem=100, width=32, hidden=4)), ("c1", dict(n_elem=64, width=128, hidden=4))]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "bf16x3", "bf16x3f"])
@pytest.mark.parametrize("name,over", GRAD_CASES)
def test_loss_and_gradients(prec, name, over):
    """Robust loss, dLOSS/dtheta and dLOSS/dlogK of the same parameters.
    Widths 32/64 with 3-4 hidden layers run on the matrix cores in fp32/bf16
    (257^2 and 101^2 nodes leave a partial last 32-node tile)."""
    say("loss_grad", prec, name, over)
    prob = problem(name, **over)
    widths = (32, 64) if prec == "bf16x3" else (32, 64, 128)
    if prec.startswith("bf16") and not (prob.width in widths and prob.hidden in (3, 4)):
        pytest.skip("bf16 network paths: widths 32/64 (bf16 and the mixed form also 128), "
                    "3-4 hidden layers")
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob)
    loss, g, gl = sc.loss_grad(with_logperm=True)
    lref, gref = orc.loss_and_grad()
    glref = orc.loss_grad_logperm()
    el = abs(loss - lref) / abs(lref)
    say(f"  loss {el:.2e}")
    tol = {"fp64": 1e-10, "fp32": 1e-4, "bf16": 1e-1, "bf16x3": 1e-4, "bf16x3f": 1e-4}[prec]
    # mixed form: loss and dlogK come from the split-bf16 forward (1e-4); the
    # network backward rounds activations and deltas to bf16 (2^-9 each, random
    # across nodes), so dtheta gets 3e-3 (measured up to 1.0e-3)
    assert el <= tol
    check("dlogK", gl, glref, tol)
    check("dtheta", g, gref, 3e-3 if prec == "bf16x3f" else tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ne,r", [(32, 2), (33, 3), (256, 2)])
def test_projection(prec, ne, r):
    say("projection", prec, ne, r)
    prob = problem("c1", n_elem=ne, degree=r)
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob)
    p = sc.project_pressure()
    pref = ads.project_nodal(orc.space, orc.u_nodal())
    check("p", p, pref, 1e-11 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nsub", [1, 10])
@pytest.mark.parametrize("ne,r,wells", [(32, 2, "pair"), (40, 3, "pair"), (128, 2, "five")])
def test_saturation_substeps(prec, nsub, ne, r, wells):
    """Each substep is one assembly plus one Kronecker mass solve; in FP32 one
    substep must meet the 1e-5 ADS criterion and ten accumulate at most ten
    such errors (1e-4)."""
    say("substeps", prec, nsub, ne, r)
    prob = problem("c1", n_elem=ne, degree=r, wells=wells)
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob)
    nb = ne + r
    s0 = np.random.default_rng(ne).uniform(0.0, 0.6, (nb, nb))
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
    tol = 1e-12 if prec == "fp64" else 1e-5 * nsub
    check("S", s_gpu, orc.s, tol)
    check("S nodal", sn_gpu, orc.s_nodal, tol)
    check("dS", s_gpu - s0, orc.s - s0, 1e-10 if prec == "fp64" else 1e-3)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-3), ("bf16x3", 5e-3),
                                      ("bf16x3f", 5e-3)])
def test_coupled_trajectory_c1(prec, tol):
    """C1 geometry: pretraining then coupled steps, fields after every step."""
    say("coupled c1", prec)
    prob = problem("c1")
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob, lr=1e-4)
    n_pre, n_steps = 500, 3
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
    hist = sc.loss_history()
    assert len(hist) == n_pre + n_steps * 100
    say(f"  loss history {rel(hist, np.array(orc.loss_history)):.3e}")
    check("hist", hist, np.array(orc.loss_history), tol)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-3), ("bf16x3", 5e-3),
                                      ("bf16x3f", 5e-3)])
def test_coupled_trajectory_c1_full(prec, tol):
    """The whole C1 configuration: 2000 pretraining iterations, then 10 coupled
    steps of 100 Adam iterations (lr 1e-4), fields compared after every step."""
    say("coupled c1 full", prec)
    prob = problem("c1")
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob, lr=1e-4)
    l_gpu = sc.pretrain_pressure(prob.pretrain_iters)
    orc.pretrain(prob.pretrain_iters)
    say(f"  pretrain loss {abs(l_gpu - orc.loss_history[-1]) / abs(orc.loss_history[-1]):.3e}")
    dt = cfl_dt(orc)
    worst = 0.0
    for k in range(prob.steps):
        sc.step(dt)
        orc.step(dt)
        p, s, sn = sc.fields()
        pr, sr, snr = orc.fields()
        say(f"  step {k}")
        for lab, a, b in (("p", p, pr), ("S", s, sr), ("S nodal", sn, snr)):
            worst = max(worst, *check(lab, a, b, tol))
    say(f"  worst {worst:.3e}")


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-3), ("bf16x3f", 5e-3)])
def test_coupled_trajectory_width128(prec, tol):
    """The wider network, 2 -> 4x128 -> 1, on the matrix cores (float32:
    one wave per SIMD, four waves per block; mixed form: eight) through
    pretraining and coupled steps on a 40^2-element grid against the oracle."""
    say("coupled width 128", prec)
    prob = problem("c1", n_elem=40, width=128, hidden=4)
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob, lr=1e-4)
    n_pre, n_steps = 300, 2
    l_gpu = sc.pretrain_pressure(n_pre)
    orc.pretrain(n_pre)
    assert abs(l_gpu - orc.loss_history[-1]) <= tol * abs(orc.loss_history[-1])
    dt = cfl_dt(orc)
    for k in range(n_steps):
        sc.step(dt)
        orc.step(dt)
        p, s, sn = sc.fields()
        pr, sr, snr = orc.fields()
        check(f"step {k}, p", p, pr, tol)
        check(f"step {k}, S", s, sr, tol)
    check("loss history", sc.loss_history(), np.array(orc.loss_history), tol)
    sc.close()
