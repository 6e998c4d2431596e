"""Model variants on the same kernels, against the FP64 oracle:

* linear relative permeabilities (exponent 1), a spatially varying porosity,
  a non-zero initial saturation and another viscosity ratio (the paper's
  model with kr = S allows these directly: eq. 5 with n = 1, phi(x));
* state export / import: a context rebuilt from another's exported state
  continues bitwise identically (checkpoint / resume);
* the inverse direction the paper names as future work: descent on log K
  driven by the adjoint dLOSS/dlog K lowers the loss for a fixed network;
* (split-bf16 forms) resume after set_state is bitwise, i.e. the fragment
  repack from theta equals the Adam kernel's in-place fragment update.
"""
import dataclasses

import numpy as np
import pytest

from helpers import check, oracle_for, problem, rel, say, scenario_for
from oracle import cfl_dt

pytestmark = pytest.mark.gpu


def _variant_problem():
    prob = problem("c1")
    n = prob.porosity.shape[0]
    x = np.linspace(0.0, 1.0, n)
    # nodal arrays are x fastest: axis 0 is y, axis 1 is x
    y2, x2 = np.meshgrid(x, x, indexing="ij")
    poro = 0.2 + 0.08 * np.sin(2.0 * np.pi * x2) * np.cos(np.pi * y2)
    nb = prob.n_elem + prob.degree
    s0 = np.random.default_rng(11).uniform(0.0, 0.3, size=(nb, nb))
    return dataclasses.replace(prob, porosity=poro, s0_coefs=s0)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-3), ("bf16x3f", 5e-3)])
def test_linear_relperm_variable_porosity(prec, tol):
    say("variant: kr = S, phi(x), S0 != 0, mu_w/mu_g = 4", prec)
    prob = _variant_problem()
    model = dict(relperm_exp=1.0, mu_g=0.25, lr=1e-4)
    sc = scenario_for(prob, prec, **model)
    orc = oracle_for(prob, **model)
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
    # the saturation really moved, and differently from the quadratic model
    assert rel(orc.s, prob.s0_coefs) > 1e-6


@pytest.mark.parametrize("prec", ["fp32", "bf16x3f"])
def test_state_export_import_resumes_bitwise(prec):
    say("checkpoint / resume", prec)
    prob = problem("c1")
    a = scenario_for(prob, prec)
    a.pretrain_pressure(50)
    dt = 1e-4
    a.step(dt)
    theta, m, v, t = a.get_state()
    _, s_coefs, _ = a.fields()
    b = scenario_for(prob, prec)
    b.pretrain_pressure(1)            # any state: everything below replaces it
    b.set_state(theta, m, v, t)
    b.set_saturation(s_coefs)
    for sc in (a, b):
        sc.step(dt)
    pa, sa, _ = a.fields()
    pb, sb, _ = b.fields()
    assert np.array_equal(pa, pb) and np.array_equal(sa, sb)
    assert np.array_equal(a.get_state()[0], b.get_state()[0])
    assert a.get_state()[3] == b.get_state()[3] == t + 100


def test_log_perm_descent_lowers_loss():
    """With the network trained on the true log K and then held fixed, Adam
    steps on log K along the adjoint gradient fit the field to that network
    pressure: from a perturbed start the loss drops by more than 20 %, below
    its value at the true field (the network after 2000 iterations is not
    the exact pressure, so other fields fit it better), and ends at its
    lowest value.  This exercises the adjoint-driven log K optimisation, not
    the recovery of the true field."""
    import torch
    from paper_2604_20731_amd.autograd import crv_loss
    say("log K descent")
    prob = problem("c1")
    sc = scenario_for(prob, "fp32")
    sc.pretrain_pressure(2000)
    theta = torch.tensor(sc.get_state()[0], dtype=torch.float64)
    l_true = float(crv_loss(theta, torch.tensor(prob.log_perm, dtype=torch.float64), sc))
    rng = np.random.default_rng(3)
    lk = torch.tensor(prob.log_perm + 0.3 * rng.standard_normal(prob.log_perm.shape),
                      dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([lk], lr=0.02)
    losses = []
    for _ in range(40):
        opt.zero_grad()
        loss = crv_loss(theta, lk, sc)
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
    say(f"  loss at true log K {l_true:.4e}; perturbed {losses[0]:.4e} -> {losses[-1]:.4e}")
    say("  " + " ".join(f"{x:.3e}" for x in losses[::5]))
    assert losses[-1] < 0.8 * losses[0] and losses[-1] < l_true
    assert losses[-1] <= 1.001 * min(losses)
