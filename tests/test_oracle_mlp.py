"""Pins of the oracle's network and Adam against torch (CPU, float64)."""
import numpy as np
import torch

from oracle import mlp
from paper_2604_20731_amd import inputs


def _torch_net(theta, dims):
    layers = []
    for (w, b) in mlp.unpack(theta, dims):
        lin = torch.nn.Linear(w.shape[1], w.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(w))
            lin.bias.copy_(torch.from_numpy(b))
        layers.append(lin)
    return layers


def _torch_fwd(layers, z):
    h = z
    for i, lin in enumerate(layers):
        h = lin(h)
        if i < len(layers) - 1:
            h = torch.tanh(h)
    return h[:, 0]


def test_forward_backward_match_torch_autograd():
    dims = mlp.layer_dims(2, 16, 3)
    theta = inputs.theta_xavier(2, 16, 3, seed=7)
    theta = theta + 0.1 * np.random.default_rng(0).standard_normal(theta.size)  # nonzero biases
    z = mlp.node_inputs(9, 2)
    g_out = np.random.default_rng(1).standard_normal(z.shape[0])
    acts = mlp.forward(theta, dims, z)
    grad = mlp.backward(theta, dims, acts, g_out)
    layers = _torch_net(theta, dims)
    out = _torch_fwd(layers, torch.from_numpy(z))
    assert np.allclose(out.detach().numpy(), acts[-1], atol=1e-13)
    (out * torch.from_numpy(g_out)).sum().backward()
    ref = np.concatenate([np.concatenate([l.weight.grad.numpy().ravel(), l.bias.grad.numpy()])
                          for l in layers])
    assert np.allclose(grad, ref, atol=1e-12)


def test_node_inputs_order():
    z = mlp.node_inputs(4, 2)
    # row index = j*5 + i, columns (x, y) mapped to [-1, 1]
    assert np.allclose(z[7], [2 * 2 / 4 - 1, 2 * 1 / 4 - 1])
    z3 = mlp.node_inputs(2, 3)
    assert np.allclose(z3[1 * 9 + 2 * 3 + 0], [-1, 1, 0])


def test_adam_matches_torch_and_first_step_closed_form():
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(50)
    grads = [rng.standard_normal(50) * s for s in (1.0, 0.1, 10.0, 1e-3)]
    opt = mlp.Adam(50, lr=1e-3)
    p = torch.nn.Parameter(torch.from_numpy(theta.copy()))
    topt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    th = theta.copy()
    for k, g in enumerate(grads):
        th_new = opt.step(th, g)
        if k == 0:
            assert np.allclose(th_new - th, -1e-3 * g / (np.abs(g) + 1e-8), atol=1e-15)
        th = th_new
        topt.zero_grad()
        p.grad = torch.from_numpy(g.copy())
        topt.step()
        assert np.allclose(th, p.detach().numpy(), atol=1e-14)
