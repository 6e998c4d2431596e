"""crv_gram_solve_noalloc (for callers that cannot allocate: its tables and
work arrays live in one fixed device array) against crv_gram_solve through a
context, on two calls in a row, the second on a smaller grid: q within the
float32 Gram-solve bar (1e-5 relative L2 and elementwise, normalised by the
largest entry), and the returned loss res . q against the same product of
the context path's q in float64.  Sizes beyond the array's limit are refused
before any device work."""
import numpy as np
import pytest

from helpers import check, say

pytestmark = pytest.mark.gpu


def _context_q(ne, res):
    from paper_2604_20731_amd import crv, inputs
    prob = inputs.make_problem("b512", seed=1, n_elem=ne, width=32)
    cfg = crv.config(dim=2, n_elem=ne, degree=2, width=32, hidden=4, precision="fp32")
    sc = crv.Scenario(cfg, prob.log_perm, prob.porosity, prob.wells, prob.theta0)
    q = sc.gram_solve(res)
    sc.close()
    return q


def test_noalloc_gram_solve_equals_context_path():
    import torch
    from paper_2604_20731_amd import crv
    for k, ne in enumerate([512, 100]):   # the largest grid, then a smaller padded one
        m = ne - 1
        rng = np.random.default_rng(40 + k)
        res = rng.standard_normal((m, m)).astype(np.float32)
        r_t = torch.from_numpy(res).cuda()
        q_t = torch.full((m, m), float("nan"), dtype=torch.float32, device="cuda")
        l_t = torch.zeros(1, dtype=torch.float64, device="cuda")
        crv.gram_solve_noalloc(ne, r_t, q_t, l_t)
        torch.cuda.synchronize()
        q = q_t.cpu().numpy().astype(np.float64)
        q_ref = _context_q(ne, res.astype(np.float64))
        say(f"call {k + 1}: n_elem {ne}")
        check("q against crv_gram_solve", q, q_ref, 1e-5)
        loss_ref = float(np.dot(res.astype(np.float64).ravel(), q_ref.ravel()))
        e = abs(float(l_t.item()) - loss_ref) / abs(loss_ref)
        say(f"  loss {l_t.item():.8e} vs {loss_ref:.8e}: rel {e:.2e}")
        assert e < 1e-5


def test_noalloc_refuses_sizes_beyond_its_array():
    import torch
    from paper_2604_20731_amd import crv
    ne = 513
    r_t = torch.zeros((ne - 1) ** 2, dtype=torch.float32, device="cuda")
    q_t = torch.zeros_like(r_t)
    with pytest.raises(crv.CrvError) as ei:
        crv.gram_solve_noalloc(ne, r_t, q_t)
    assert ei.value.status == crv.CRV_EINVAL
