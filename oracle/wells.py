"""Well discs -> nodal source arrays (oracle, test infrastructure).

The paper models injection as a disc-shaped source of given strength at the
domain centre (results, simulation set-up).  Reading used for the generated
scenarios: each well w = (x_w, y_w, r_w) covers the nodes with
(x - x_w)^2 + (y - y_w)^2 <= R^2 (in 3D a vertical cylinder over the interior
z nodes), and spreads its rate evenly over them so that h^d sum_p q_p = r_w.
Injectors (r > 0) and producers (r < 0) are kept in separate arrays: the
pressure uses their sum, the saturation update uses the injector rate as the
gas source and the producer rate times the gas fractional flow.

The disc test is done in float64 as written below; a disc reaching a boundary
node or covering no node is rejected.
"""
from __future__ import annotations

import numpy as np


def nodal_sources(wells: np.ndarray, n_elem: int, dim: int, radius: float):
    n = n_elem + 1
    h = 1.0 / n_elem
    q_inj = np.zeros((n,) * dim)
    q_prod = np.zeros((n,) * dim)
    i = np.arange(n)
    xs = i / n_elem
    for xw, yw, rate in np.asarray(wells, dtype=np.float64):
        dx = xs - xw
        dy = xs - yw
        dx2 = dx * dx
        dy2 = dy * dy
        disc = (dy2[:, None] + dx2[None, :]) <= radius * radius   # (y, x)
        if dim == 2:
            mask = disc
        else:
            mask = np.zeros((n, n, n), dtype=bool)
            mask[1:n - 1] = disc[None, :, :]
        cnt = int(mask.sum())
        if cnt == 0:
            raise ValueError("well covers no node")
        bnd = np.ones((n,) * dim, dtype=bool)
        bnd[tuple(slice(1, n - 1) for _ in range(dim))] = False
        if np.any(mask & bnd):
            raise ValueError("well reaches the boundary")
        val = rate / (h ** dim * cnt)
        if rate >= 0:
            q_inj[mask] += val
        else:
            q_prod[mask] += val
    return q_inj, q_prod
