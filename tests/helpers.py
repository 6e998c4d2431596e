"""Shared builders for the GPU parity tests: the same seeded Problem feeds the
HIP scenario and the FP64 oracle (which share no code)."""
import math

import numpy as np

from paper_2604_20731_amd import inputs


def rel(a, b):
    """Relative L2 error |a - b| / |b|."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def maxrel(a, b):
    """Elementwise error normalised by the field's scale, max|a - b| / max|b|.
    Beside the relative L2 error it catches errors confined to a few entries
    (one wrong boundary row, a padded tile), which an L2 norm over the whole
    field dilutes."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.size == 0:
        return 0.0
    mb = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0))


def check(label, a, b, tol, max_tol=None):
    """Print both errors and require rel-L2 < tol and max-rel < max_tol (tol
    unless given).  Returns (rel-L2, max-rel)."""
    e2, em = rel(a, b), maxrel(a, b)
    mt = tol if max_tol is None else max_tol
    say(f"  {label}: relL2 {e2:.2e} max {em:.2e} (tol {tol:.0e}/{mt:.0e})")
    assert e2 < tol and em < mt, (label, e2, em, tol, mt)
    return e2, em


def problem(name, seed=0, **over):
    return inputs.make_problem(name, seed=seed, **over)


def oracle_for(prob, **kw):
    from oracle import Oracle
    return Oracle(prob.dim, prob.n_elem, prob.degree, prob.width, prob.hidden, prob.log_perm,
                  prob.porosity, prob.wells, prob.theta0, prob.s0_coefs, **kw)


def scenario_for(prob, precision, **kw):
    from paper_2604_20731_amd import crv
    return crv.scenario_from_problem(prob, precision, **kw)


def say(*a):
    print(*a, flush=True)


def splitmix64(seed, k):
    """Output k of SplitMix64 started at state seed (Steele, Lea and Flood,
    OOPSLA 2014), written out from its definition."""
    m = (1 << 64) - 1
    z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def default_theta(dim, width, hidden, seed):
    """The library's seeded default parameters: Xavier-uniform weights from
    splitmix64 outputs in layout order (top 53 bits), zero biases."""
    d = [dim] + [width] * hidden + [1]
    out, k = [], 0
    for i in range(len(d) - 1):
        a = math.sqrt(6.0 / (d[i] + d[i + 1]))
        for _ in range(d[i] * d[i + 1]):
            u = (splitmix64(seed, k) >> 11) * 2.0 ** -53
            out.append(a * (2.0 * u - 1.0))
            k += 1
        out += [0.0] * d[i + 1]
    return np.array(out)
