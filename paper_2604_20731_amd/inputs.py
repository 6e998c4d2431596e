"""Seeded synthetic inputs for the hybrid CO2 solver.

This module only draws random problem data: log-permeability fields, porosity,
well lists, initial network weights and the scenario mix of the serving
workload.  It holds none of the solver's arithmetic, so both the HIP path and
the FP64 oracle can consume the same arrays without sharing any numerics.

The paper runs on private porosity/permeability maps (Results, simulation set-up)
that survive only as figures; these generators stand in for them with the same
structure: a smooth heterogeneous log-permeability, uniform porosity and disc
shaped injection/production sources.

Array conventions (shared by every consumer):
  * nodal arrays on the (N+1)^d collocation nodes x_i = i/N, numpy shape
    (ny, nx) or (nz, ny, nx), C order, so x is the fastest index;
  * wells are rows (x, y, rate); rate > 0 injects gas, rate < 0 produces;
  * network parameters are one flat float64 vector, layer by layer,
    W_l (out x in, row-major) followed by b_l (out).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


def _rng(seed: int, stream: int) -> np.random.Generator:
    """Independent PCG64 stream per (seed, purpose)."""
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


_STREAM_PERM, _STREAM_WELLS, _STREAM_THETA, _STREAM_BANDS, _STREAM_MIX = 1, 2, 3, 4, 5


def _sqexp_factor(n_nodes: int, ell: float) -> np.ndarray:
    """F with F F^T = exp(-(x-x')^2 / (2 ell^2)) on the nodes x = linspace(0,1,n)."""
    x = np.linspace(0.0, 1.0, n_nodes)
    c = np.exp(-((x[:, None] - x[None, :]) ** 2) / (2.0 * ell * ell))
    lam, q = np.linalg.eigh(c)
    lam = np.clip(lam, 0.0, None)
    return q * np.sqrt(lam)[None, :]


def grf(n_elem: int, dim: int, ell: float, sigma: float, seed: int,
        stream: int = _STREAM_PERM) -> np.ndarray:
    """Zero-mean Gaussian random field with covariance
    sigma^2 exp(-|x-x'|^2 / (2 ell^2)) on the (N+1)^dim nodes, sampled exactly
    through the separability of the squared-exponential kernel."""
    n = n_elem + 1
    f = _sqexp_factor(n, ell)
    xi = _rng(seed, stream).standard_normal((n,) * dim)
    if dim == 2:
        return sigma * (f @ xi @ f.T)
    if dim == 3:
        return sigma * np.einsum("kc,jb,ia,cba->kji", f, f, f, xi, optimize=True)
    raise ValueError("dim must be 2 or 3")


def layered(n_elem: int, seed: int, n_bands: int = 8, offset: float = 2.0,
            noise_sigma: float = 0.5, noise_ell: float = 0.05) -> np.ndarray:
    """2D layered log-permeability: n_bands horizontal bands with offsets
    U(-offset, offset) plus a GRF of standard deviation noise_sigma."""
    n = n_elem + 1
    off = _rng(seed, _STREAM_BANDS).uniform(-offset, offset, size=n_bands)
    y = np.arange(n) / n_elem
    band = np.minimum(np.floor(n_bands * y).astype(np.int64), n_bands - 1)
    base = np.repeat(off[band][:, None], n, axis=1)
    return base + grf(n_elem, 2, noise_ell, noise_sigma, seed)


def porosity(n_elem: int, dim: int, value: float = 0.2) -> np.ndarray:
    return np.full((n_elem + 1,) * dim, float(value))


def wells_fixed_pair() -> np.ndarray:
    """One injector at (0.25, 0.5) and one producer at (0.75, 0.5), rate 1."""
    return np.array([[0.25, 0.5, 1.0], [0.75, 0.5, -1.0]])


def wells_balanced(n_wells: int, seed: int, lo: float = 0.1, hi: float = 0.9) -> np.ndarray:
    """n wells at uniform positions in [lo,hi]^2 with rates U(-1,1), shifted to
    sum to zero and scaled so the largest |rate| is 1.  A single well is an
    injector of rate 1."""
    g = _rng(seed, _STREAM_WELLS)
    pos = g.uniform(lo, hi, size=(n_wells, 2))
    if n_wells == 1:
        return np.array([[pos[0, 0], pos[0, 1], 1.0]])
    rate = g.uniform(-1.0, 1.0, size=n_wells)
    rate = rate - rate.mean()
    rate = rate / np.abs(rate).max()
    return np.column_stack([pos, rate])


def wells_injectors(n_wells: int, seed: int, lo: float = 0.1, hi: float = 0.9) -> np.ndarray:
    g = _rng(seed, _STREAM_WELLS)
    pos = g.uniform(lo, hi, size=(n_wells, 2))
    return np.column_stack([pos, np.ones(n_wells)])


def layer_dims(dim: int, width: int, hidden: int) -> List[int]:
    return [dim] + [width] * hidden + [1]


def n_params(dim: int, width: int, hidden: int) -> int:
    d = layer_dims(dim, width, hidden)
    return sum(d[i + 1] * d[i] + d[i + 1] for i in range(len(d) - 1))


def theta_xavier(dim: int, width: int, hidden: int, seed: int) -> np.ndarray:
    """Xavier-uniform weights, zero biases, flat layout W_l then b_l per layer."""
    g = _rng(seed, _STREAM_THETA)
    d = layer_dims(dim, width, hidden)
    parts = []
    for i in range(len(d) - 1):
        fan_in, fan_out = d[i], d[i + 1]
        a = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(g.uniform(-a, a, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


@dataclasses.dataclass
class Problem:
    """Everything a scenario needs besides the solver configuration."""
    name: str
    dim: int
    n_elem: int
    degree: int
    width: int
    hidden: int
    log_perm: np.ndarray
    porosity: np.ndarray
    wells: np.ndarray
    theta0: np.ndarray
    pretrain_iters: int
    steps: int
    precision: str = "fp32"      # "fp64" | "fp32" | "bf16"
    seed: int = 0
    s0_coefs: Optional[np.ndarray] = None


def make_problem(name: str, seed: int = 0, **over) -> Problem:
    """The named workloads:

    c1    2D, 32 quadratic elements, 33^2 nodes, 2->3x32->1, FP64 debug parity,
          GRF l=0.1, injector/producer pair, 2000 pretraining, 10 steps.
    c2    2D, 256 quadratic elements, 257^2 nodes, 2->4x64->1, FP32, GRF l=0.05,
          5 balanced wells, 50 steps.
    b512  2D, 512 quadratic elements, 513^2 nodes, 2->4x64->1, GRF l=0.05,
          5 balanced wells (the throughput workload).
    c3    2D, 1024 cubic elements, 1025^2 nodes, 2->4x128->1, BF16 MLP,
          layered log-permeability, 5 balanced wells, 20 steps.
    c5    3D, 128 quadratic elements, 129^3 nodes, 3->4x128->1, BF16 MLP,
          GRF l=0.1, two vertical injectors, 10 steps.
    tiny  2D, 8 quadratic elements, 2->2x16->1 (unit tests).
    """
    presets = {
        "tiny": dict(dim=2, n_elem=8, degree=2, width=16, hidden=2, ell=0.2, wells="pair",
                     pretrain_iters=20, steps=2, precision="fp64"),
        "c1": dict(dim=2, n_elem=32, degree=2, width=32, hidden=3, ell=0.1, wells="pair",
                   pretrain_iters=2000, steps=10, precision="fp64"),
        "c2": dict(dim=2, n_elem=256, degree=2, width=64, hidden=4, ell=0.05, wells="five",
                   pretrain_iters=2000, steps=50, precision="fp32"),
        "b512": dict(dim=2, n_elem=512, degree=2, width=64, hidden=4, ell=0.05, wells="five",
                     pretrain_iters=2000, steps=20, precision="fp32"),
        "c3": dict(dim=2, n_elem=1024, degree=3, width=128, hidden=4, ell=None, wells="five",
                   pretrain_iters=2000, steps=20, precision="bf16"),
        "c5": dict(dim=3, n_elem=128, degree=2, width=128, hidden=4, ell=0.1, wells="inj2",
                   pretrain_iters=2000, steps=10, precision="bf16"),
    }
    p = dict(presets[name])
    p.update(over)
    dim, ne = p["dim"], p["n_elem"]
    if p["ell"] is None:
        logk = layered(ne, seed)
    else:
        logk = grf(ne, dim, p["ell"], 1.0, seed)
    w = p["wells"]
    if isinstance(w, np.ndarray):
        wells = w
    elif w == "pair":
        wells = wells_fixed_pair()
    elif w == "five":
        wells = wells_balanced(5, seed)
    elif w == "inj2":
        wells = wells_injectors(2, seed)
    else:
        raise ValueError(w)
    theta = theta_xavier(dim, p["width"], p["hidden"], seed)
    return Problem(name=name, dim=dim, n_elem=ne, degree=p["degree"], width=p["width"],
                   hidden=p["hidden"], log_perm=logk, porosity=porosity(ne, dim),
                   wells=wells, theta0=theta, pretrain_iters=p["pretrain_iters"],
                   steps=p["steps"], precision=p["precision"], seed=seed)


@dataclasses.dataclass
class Arrival:
    t: float
    n_elem: int
    width: int
    seed: int
    n_wells: int


def serving_mix(n: int = 64, mean_gap_s: float = 0.05, seed: int = 0,
                grids=(64, 128, 256, 512), widths=(64, 128)) -> List[Arrival]:
    """Poisson arrivals (exponential gaps of mean mean_gap_s), grid and width
    drawn uniformly, 1-8 wells, one seed per scenario."""
    g = _rng(seed, _STREAM_MIX)
    t = np.cumsum(g.exponential(mean_gap_s, size=n))
    out = []
    for k in range(n):
        out.append(Arrival(t=float(t[k]), n_elem=int(g.choice(grids)),
                           width=int(g.choice(widths)), seed=int(1000 + k),
                           n_wells=int(g.integers(1, 9))))
    return out
