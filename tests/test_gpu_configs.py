"""The full-size configurations against the FP64 oracle (each oracle call is
seconds to half a minute):

* 257^2 FP32 (2 -> 4x64 -> 1, five wells): teacher-forced coupled steps --
  before each step the oracle takes the GPU's network, Adam moments, step
  count and saturation, then both run one full step (projection, ten
  substeps, refresh, 100 Adam iterations) and the fields are compared.
* 1025^2 cubic, 2 -> 4x128 -> 1, layered log-permeability: loss and
  gradients at the GPU's parameters after a short pretraining, the network
  pressure on the 2x-coarsened check grid, and ten FP32 saturation substeps.
  FP32 network (per-node kernels at width 128) to 1e-4; the plain bf16 network
  is run with its error reported against the documented bf16 bound.
"""
import numpy as np
import pytest

from helpers import oracle_for, problem, rel, say, scenario_for
from oracle import ads, bspline, cfl_dt

pytestmark = pytest.mark.gpu


def _take_state(orc, sc):
    th, m, v, t = sc.get_state()
    _, s, _ = sc.fields()
    orc.theta = th.copy()
    orc.adam.m, orc.adam.v, orc.adam.t = m.copy(), v.copy(), int(t)
    orc.s = s.copy()
    orc.refresh()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-3), ("bf16x3", 5e-3), ("bf16x3f", 5e-3)])
def test_c2_teacher_forced_steps(prec, tol):
    """2 -> 4x64 -> 1 (the network of the 512^2 throughput workload)."""
    say("c2 257^2 teacher-forced steps", prec)
    prob = problem("c2")
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob)
    dt = cfl_dt(orc)
    sc.pretrain_pressure(300)
    for k in range(2):
        _take_state(orc, sc)
        sc.step(dt)
        orc.step(dt)
        p, s, sn = sc.fields()
        pr, sr, snr = orc.fields()
        e = (rel(p, pr), rel(s, sr), rel(sn, snr))
        say(f"  step {k}: p {e[0]:.2e}  S {e[1]:.2e}  S nodal {e[2]:.2e}")
        assert max(e) < tol


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 0.15), ("bf16x3f", 5e-3)])
def test_c3_network_loss_and_fields(prec, tol):
    """bf16: products of bf16-rounded operands; the 0.15 bound on the network
    pressure and dtheta is the plain-bf16 error documented for this network
    shape (the split-bf16 form exists for widths up to 64).  The loss, a small
    difference of large terms (RES = A u - h^2 q), is reported but not bounded
    in bf16: a 7% error in u moves it by O(1).  The mixed form (split-bf16
    forward, bf16 backward products on split weights) is held to the 5e-3
    field tolerance."""
    say("c3 1025^2 cubic", prec)
    prob = problem("c3")
    sc = scenario_for(prob, prec)
    sc.pretrain_pressure(20)
    th = sc.get_state()[0]
    orc = oracle_for(prob)
    loss, g = sc.loss_grad()
    lref, gref = orc.loss_and_grad(th)
    p = sc.fields()[0]
    pref = orc.u_nodal(th)
    e = dict(loss=abs(loss - lref) / abs(lref), dtheta=rel(g, gref),
             p_coarse=rel(p[::2, ::2], pref[::2, ::2]))
    say("  " + "  ".join(f"{k} {v:.2e}" for k, v in e.items()))
    if prec == "bf16":
        e.pop("loss")
    assert all(v < tol for v in e.values()), e


@pytest.mark.timeout(900)
def test_c3_saturation_substeps():
    """Ten FP32 substeps at 1028^2 cubic coefficients with tau a tenth of the
    CFL step of the network pressure (beyond CFL the explicit update amplifies
    any rounding difference); tolerance from the conditioning of the cubic
    mass matrix (cond(M_1)^2 2^-24 per substep)."""
    say("c3 substeps fp32")
    prob = problem("c3")
    sc = scenario_for(prob, "fp32")
    orc = oracle_for(prob)
    nb = prob.n_elem + prob.degree
    s0 = np.random.default_rng(3).uniform(0.0, 0.6, (nb, nb))
    sc.set_saturation(s0)
    orc.s = s0.copy()
    orc.refresh()
    from paper_2604_20731_amd.serve import cfl_dt as cfl_from_pressure
    tau = 0.1 * cfl_from_pressure(sc.fields()[0], prob.log_perm, prob.porosity, prob.n_elem)
    nsub = 10
    sc.saturation_substeps(tau, nsub)
    pproj = ads.project_nodal(orc.space, orc.u_nodal())
    for _ in range(nsub):
        orc.s = ads.saturation_substep(orc.space, orc.s, pproj, orc.perm, orc.poro, orc.q_inj,
                                       orc.q_prod, tau, orc.mu_w, orc.mu_g, orc.n_exp)
    orc.refresh()
    _, s_gpu, sn_gpu = sc.fields()
    tol = nsub * max(1e-5, np.linalg.cond(bspline.mass_1d(prob.n_elem, prob.degree)) ** 2 * 2.0 ** -24)
    e = (rel(s_gpu, orc.s), rel(sn_gpu, orc.s_nodal), rel(s_gpu - s0, orc.s - s0))
    say(f"  S {e[0]:.2e}  S nodal {e[1]:.2e}  increment {e[2]:.2e}  (tol {tol:.1e})")
    # the increment is small at this tau: its error is the M^-1 (M S) rounding
    # of S itself (bounded above), so it is reported, not bounded separately
    assert e[0] < tol and e[1] < tol
