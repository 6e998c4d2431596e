"""Fully connected tanh network and Adam (oracle, test infrastructure).

The paper replaces the pressure by the output of a neural network evaluated
at the collocation nodes but does not state the architecture; the workloads
use d -> hidden x width (tanh) -> 1 with a linear output.  The network input is
the node position mapped to [-1, 1]^d, and the output is multiplied by the
interior indicator so the trial function vanishes on the boundary.  Training
minimises the robust loss with Adam (results: pretraining, then 100 iterations
per pressure update), with moments and step count kept across updates.

Parameter layout: one flat vector, per layer W (out x in, row-major) then b.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def layer_dims(dim: int, width: int, hidden: int) -> List[int]:
    return [dim] + [width] * hidden + [1]


def unpack(theta: np.ndarray, dims: Sequence[int]) -> List[Tuple[np.ndarray, np.ndarray]]:
    out, o = [], 0
    for i in range(len(dims) - 1):
        fi, fo = dims[i], dims[i + 1]
        w = theta[o:o + fo * fi].reshape(fo, fi)
        o += fo * fi
        b = theta[o:o + fo]
        o += fo
        out.append((w, b))
    assert o == theta.size
    return out


def node_inputs(n_elem: int, dim: int) -> np.ndarray:
    """Network inputs 2x - 1 at every node, rows in C order of the nodal array,
    columns (x, y[, z])."""
    c = 2.0 * (np.arange(n_elem + 1) / n_elem) - 1.0
    grids = np.meshgrid(*([c] * dim), indexing="ij")  # axis order (z,)y,x
    cols = [g.ravel() for g in reversed(grids)]        # x first
    return np.column_stack(cols)


def forward(theta, dims, z):
    """Activations of every layer; the last entry is the output (npts,)."""
    layers = unpack(theta, dims)
    acts = [z]
    h = z
    for li, (w, b) in enumerate(layers):
        y = h @ w.T + b
        h = y if li == len(layers) - 1 else np.tanh(y)
        acts.append(h)
    acts[-1] = acts[-1][:, 0]
    return acts


def backward(theta, dims, acts, g_out) -> np.ndarray:
    """Gradient of sum_p g_out[p] * NN(z_p) with respect to theta (flat)."""
    layers = unpack(theta, dims)
    grads = [None] * len(layers)
    delta = g_out[:, None]
    for li in reversed(range(len(layers))):
        w, _ = layers[li]
        h_in = acts[li]
        grads[li] = (delta.T @ h_in, delta.sum(axis=0))
        if li > 0:
            delta = (delta @ w) * (1.0 - acts[li] ** 2)
    return np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])


class Adam:
    """Adam: m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
    theta <- theta - lr * mhat / (sqrt(vhat) + eps) with bias-corrected
    mhat = m / (1 - b1^t), vhat = v / (1 - b2^t)."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)
