"""Shared builders for the GPU parity tests: the same seeded Problem feeds the
HIP scenario and the FP64 oracle (which share no code)."""
import numpy as np

from paper_2604_20731_amd import inputs


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


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
