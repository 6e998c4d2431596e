"""Writes the stored expected values of the configuration-scale GPU tests.

Calls only the FP64 oracle (oracle/) and the seeded input generators; no
value comes from the HIP path.  Each file records the command that made it.

    python tests/golden/make_goldens.py c2          # c2_trajectory.npz
    python tests/golden/make_goldens.py divergence  # c1_divergence.npz

c2: the 257^2 configuration (256 quadratic elements, 2 -> 4x64 -> 1, GRF
    l = 0.05, five balanced wells, seed 0), 2000 pretraining iterations and
    10 coupled steps of 100 Adam iterations (IGA-ADS-CRVPINN algorithm,
    steps 2-8), lr 1e-4.  Stored after the pretraining and after steps 1, 2,
    5 and 10: nodal network pressure and saturation coefficients (float32),
    plus the whole loss history and dt (CFL 0.5 from the direct solve of the
    initial pressure system).
divergence: how two FP64 runs of the 33^2 configuration that differ only by
    a relative 1e-12 perturbation of the initial weights drift apart, per Adam
    iteration (2000 pretraining + 10 x 100), at the configurations' lr 1e-3
    and at 1e-4: the run-to-run spread that any parity bound on a trajectory
    has to sit above.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import Oracle, cfl_dt  # noqa: E402
from paper_2604_20731_amd import inputs  # noqa: E402


def _oracle(prob, theta0=None, lr=1e-4):
    return Oracle(prob.dim, prob.n_elem, prob.degree, prob.width, prob.hidden, prob.log_perm,
                  prob.porosity, prob.wells, prob.theta0 if theta0 is None else theta0,
                  prob.s0_coefs, lr=lr)


def _log(msg):
    print(f"[golden] {msg}", flush=True)


def make_c2(out_dir, pretrain=2000, steps=10, checkpoints=(1, 2, 5, 10)):
    prob = inputs.make_problem("c2", seed=0)
    orc = _oracle(prob)
    dt = cfl_dt(orc)
    t0 = time.time()
    for k in range(0, pretrain, 100):
        orc.train(min(100, pretrain - k))
        _log(f"c2 pretraining {k + 100}/{pretrain}  loss {orc.loss_history[-1]:.6e}  "
             f"{time.time() - t0:.0f} s")
    store = {}

    def keep(tag):
        u, s, _ = orc.fields()
        store[f"u_{tag}"] = u.astype(np.float32)
        store[f"s_{tag}"] = s.astype(np.float32)

    keep("pre")
    for k in range(1, steps + 1):
        orc.step(dt)
        _log(f"c2 step {k}/{steps}  loss {orc.loss_history[-1]:.6e}  {time.time() - t0:.0f} s")
        if k in checkpoints:
            keep(f"step{k}")
    path = os.path.join(out_dir, "c2_trajectory.npz")
    np.savez_compressed(path, dt=dt, pretrain=pretrain, steps=steps,
                        checkpoints=np.array(checkpoints), loss=np.array(orc.loss_history),
                        lr=1e-4, command="python tests/golden/make_goldens.py c2", **store)
    _log(f"wrote {path}")


def make_divergence(out_dir, pretrain=2000, steps=10):
    prob = inputs.make_problem("c1", seed=0)
    rng = np.random.default_rng(12345)
    th1 = prob.theta0 * (1.0 + 1e-12 * rng.standard_normal(prob.theta0.size))
    curves = {}
    for lr in (1e-3, 1e-4):
        a, b = _oracle(prob, lr=lr), _oracle(prob, th1, lr=lr)
        dt = cfl_dt(a)
        curve = []

        def rec():
            ua, ub = a.u_nodal(), b.u_nodal()
            curve.append(np.linalg.norm(ua - ub) / np.linalg.norm(ua))

        for _ in range(pretrain):
            a.train(1)
            b.train(1)
            rec()
        for k in range(steps):
            a.adam_iters = b.adam_iters = 1
            a.step(dt)
            b.step(dt)
            rec()
            for _ in range(99):
                a.train(1)
                b.train(1)
                rec()
        curves[f"lr{lr:g}"] = np.array(curve)
        _log(f"divergence lr {lr:g}: after pretraining {curve[pretrain - 1]:.2e}, "
             f"at the end {curve[-1]:.2e}, largest {max(curve):.2e}")
    path = os.path.join(out_dir, "c1_divergence.npz")
    np.savez_compressed(path, perturbation=1e-12, pretrain=pretrain, steps=steps,
                        command="python tests/golden/make_goldens.py divergence", **curves)
    _log(f"wrote {path}")


if __name__ == "__main__":
    out = os.environ.get("GOLDEN_OUT", HERE)
    os.makedirs(out, exist_ok=True)
    for what in sys.argv[1:] or ["c2", "divergence"]:
        {"c2": make_c2, "divergence": make_divergence}[what](out)
