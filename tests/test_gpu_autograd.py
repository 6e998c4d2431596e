"""Differentiation form: torch autograd through the libcrv loss (CRVLoss)
against the oracle's analytic gradients (themselves pinned to central
differences on the CPU), at parameters and log K away from the initial
ones.  Relative errors over 32 seeded coordinates and over the whole
vectors."""
import numpy as np
import pytest
import torch

from helpers import maxrel, oracle_for, problem, rel, say, scenario_for

pytestmark = pytest.mark.gpu

WELLS3 = np.array([[0.25, 0.25, 1.0], [0.75, 0.75, -1.0]])


def _check(prob, prec, tol, n_coords=32, tol_dtheta=None):
    from paper_2604_20731_amd.autograd import crv_loss
    sc = scenario_for(prob, prec)
    orc = oracle_for(prob)
    rng = np.random.default_rng(7)
    th = prob.theta0 + 0.05 * rng.standard_normal(prob.theta0.size)
    lk = prob.log_perm + 0.1 * rng.standard_normal(prob.log_perm.shape)
    t_before = sc.get_state()[3]
    theta = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    log_perm = torch.tensor(lk, dtype=torch.float64, requires_grad=True)
    loss = crv_loss(theta, log_perm, sc)
    (2.0 * loss).backward()          # the incoming gradient scales both
    orc.perm = np.exp(lk)
    orc.refresh()
    lref, gref = orc.loss_and_grad(th)
    glref = orc.loss_grad_logperm(th)
    g = theta.grad.numpy() / 2.0
    gl = log_perm.grad.numpy() / 2.0
    it = rng.choice(th.size, size=n_coords, replace=False)
    ik = rng.choice(lk.size, size=n_coords, replace=False)
    e = dict(loss=abs(float(loss.detach()) - lref) / abs(lref), dtheta32=rel(g[it], gref[it]),
             dlogK32=rel(gl.ravel()[ik], glref.ravel()[ik]), dtheta=rel(g, gref),
             dlogK=rel(gl, glref), dtheta_max=maxrel(g, gref), dlogK_max=maxrel(gl, glref))
    say("  " + "  ".join(f"{k} {v:.2e}" for k, v in e.items()))
    tt = tol if tol_dtheta is None else tol_dtheta
    assert all(v < (tt if k.startswith("dtheta") else tol) for k, v in e.items()), e
    assert sc.get_state()[3] == t_before      # training state untouched


@pytest.mark.parametrize("prec,width,tol", [("fp64", 16, 1e-10), ("fp32", 16, 1e-4),
                                            ("fp32", 32, 1e-4), ("bf16x3", 32, 1e-4)])
def test_autograd_17cubed(prec, width, tol):
    """17^3 nodes, 4 hidden layers (matrix cores for width 32)."""
    say("autograd 17^3", prec, width)
    prob = problem("c5", n_elem=16, width=width, hidden=4 if width == 32 else 2, wells=WELLS3)
    _check(prob, prec, tol)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_autograd_2d(prec, tol):
    say("autograd 2D c1", prec)
    _check(problem("c1"), prec, tol)


@pytest.mark.timeout(600)
def test_autograd_c5_full():
    """The 3D workload at full size: 129^3 nodes, 3->4x128->1, two vertical
    injectors, FP32 network."""
    say("autograd c5 129^3 fp32")
    _check(problem("c5"), "fp32", 1e-4)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,tol,tol_dtheta", [("bf16x3f", 1e-4, 3e-3), ("bf16", 1e-1, 1e-1)])
def test_autograd_c5_full_bf16(prec, tol, tol_dtheta):
    """The same full-size 3D workload with the network on bf16 matrix cores:
    the mixed form (split-bf16 forward, so loss and dlogK keep 1e-4; bf16
    activations and deltas in the backward, dtheta 3e-3) and plain bf16
    (products of bf16-rounded operands, error about 2^-9 per product through
    four layers: the documented 1e-1 bound of that form)."""
    say("autograd c5 129^3", prec)
    _check(problem("c5"), prec, tol, tol_dtheta=tol_dtheta)


def _f32_inputs(prob, seed=11):
    rng = np.random.default_rng(seed)
    th = (prob.theta0 + 0.05 * rng.standard_normal(prob.theta0.size)).astype(np.float32)
    lk = (prob.log_perm + 0.1 * rng.standard_normal(prob.log_perm.shape)).astype(np.float32)
    return th, lk


@pytest.mark.parametrize("name,prec,over,cfg", [
    ("c1", "fp32", {}, {}),
    ("c2", "bf16x3f", {}, {}),
    ("c5", "fp32", dict(n_elem=16, width=32, hidden=4, wells=WELLS3), {}),
    ("c1", "bf16x3f", {}, dict(gravity=2.0, rho_w=1.2, rho_g=0.4, boundary_factor=1)),
])
@pytest.mark.parametrize("own_stream", [False, True])
def test_device_arrays_match_host_arrays(name, prec, over, cfg, own_stream):
    """crv_set_params_device + crv_loss_grad_device (the autograd path for
    CUDA tensors) give what crv_set_state/crv_set_log_perm + crv_loss_grad
    give on the same float32 values: the same kernels on the same inputs,
    with K = exp(log K) rounded once from float64 on both sides.  With
    own_stream the scenario runs on a stream of its own while the tensors
    live on the current one.  The last case adds gravity (the right-hand side
    term of dLOSS/dlogK) and the distance trial factor."""
    from paper_2604_20731_amd.autograd import crv_loss
    say("device-array loss_grad", name, prec, "own stream" if own_stream else "current stream")
    prob = problem(name, **over)
    kw = dict(stream=torch.cuda.Stream()) if own_stream else {}
    sc = scenario_for(prob, prec, **kw, **cfg)
    th, lk = _f32_inputs(prob)
    t_before = sc.get_state()[3]
    sc.set_theta(th.astype(np.float64))
    sc.set_log_perm(lk.astype(np.float64))
    l_h, g_h, gl_h = sc.loss_grad(with_logperm=True)
    sc.set_theta(prob.theta0)           # the device call must replace both again
    sc.set_log_perm(prob.log_perm)
    theta = torch.tensor(th, device="cuda:0", requires_grad=True)
    log_perm = torch.tensor(lk, device="cuda:0", requires_grad=True)
    loss = crv_loss(theta, log_perm, sc)
    loss.backward()
    g = theta.grad.double().cpu().numpy()
    gl = log_perm.grad.double().cpu().numpy()
    e = dict(loss=abs(float(loss.detach()) - l_h) / abs(l_h), dtheta=rel(g, g_h), dlogK=rel(gl, gl_h),
             dtheta_max=maxrel(g, g_h), dlogK_max=maxrel(gl, gl_h))
    say("  " + "  ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert all(v <= 1e-6 for v in e.values()), e
    assert sc.get_state()[3] == t_before
    # the host path reads back what the device call installed
    assert np.array_equal(sc.get_state()[0], th.astype(np.float64))
    assert np.array_equal(sc.log_perm(), lk.astype(np.float64))
    sc.close()


def test_device_array_errors():
    """Non-finite log K is rejected before anything changes; host memory
    and float64 contexts are rejected; wrong sizes are caught in Python."""
    import ctypes as C
    from paper_2604_20731_amd import crv
    say("device-array error paths")
    prob = problem("c1")
    sc = scenario_for(prob, "fp32")
    l0, g0 = sc.loss_grad()
    bad = torch.tensor(prob.log_perm.ravel(), dtype=torch.float32, device="cuda:0")
    bad[5] = float("nan")
    with pytest.raises(crv.CrvError, match="non-finite"):
        sc.set_params_device(log_perm=bad)
    l1, g1 = sc.loss_grad()
    assert l1 == l0 and np.array_equal(g1, g0)
    host = torch.zeros(sc.P, dtype=torch.float32)
    st = crv.LIB.crv_loss_grad_device(sc.ctx, None, C.c_void_p(host.data_ptr()), None)
    assert st == -1 and b"device memory" in crv.LIB.crv_last_error()
    st = crv.LIB.crv_set_params_device(sc.ctx, C.c_void_p(host.data_ptr()), None)
    assert st == -1
    with pytest.raises(ValueError):
        sc.set_params_device(theta=torch.zeros(sc.P + 1, device="cuda:0"))
    l2, _ = sc.loss_grad()
    assert l2 == l0
    sc.close()
    sc64 = scenario_for(prob, "fp64")
    d = torch.zeros(sc64.P, dtype=torch.float32, device="cuda:0")
    st = crv.LIB.crv_loss_grad_device(sc64.ctx, None, C.c_void_p(d.data_ptr()), None)
    assert st == -1 and b"float32 context" in crv.LIB.crv_last_error()
    sc64.close()
