// Adjoint of the collocation residual at one node, shared by the adjoint
// kernel and the fused network backward (derived from eq. 25 and 27): with
// q~ the Gram-solved residual zero-extended to the boundary,
//   g_u(p) = 2 h^(d-2) sum_dir [alpha_{p-e} (q~_p - q~_{p-e}) - alpha_p (q~_{p+e} - q~_p)]
// at interior nodes and 0 on the boundary (the trial functions vanish there).
// q and the interior arrays are padded to pitch mp per axis.
#pragma once
#include "common.h"

namespace crv {

template <typename Real>
__device__ inline Real q_ext(const Real* q, const Geom& g, int i, int j, int k) {
  const bool in = i >= 1 && i <= g.m && j >= 1 && j <= g.m && (g.dim == 2 || (k >= 1 && k <= g.m));
  const int64_t kk = g.dim == 3 ? int64_t(k - 1) : 0;
  return in ? q[(kk * g.mp + (j - 1)) * g.mp + (i - 1)] : Real(0);
}

// g_u at node p; *iq receives the padded interior index of p (or -1 on the boundary)
template <typename Real, int DIM>
__device__ inline Real adjoint_at(const Geom& g, const Real* __restrict__ q,
                                  const Real* __restrict__ alpha, int64_t p, int64_t* iq) {
  const int64_t n = g.n;
  int i, j, k;
  node_ijk<DIM>(p, int(n), &i, &j, &k);
  if (DIM == 2) k = 1;
  const bool in = i >= 1 && i <= g.m && j >= 1 && j <= g.m && (DIM == 2 || (k >= 1 && k <= g.m));
  if (!in) {
    *iq = -1;
    return Real(0);
  }
  *iq = ((DIM == 3 ? int64_t(k - 1) : 0) * g.mp + (j - 1)) * g.mp + (i - 1);
  const Real qp = q[*iq], ap = alpha[p];
  Real s = alpha[p - 1] * (qp - q_ext(q, g, i - 1, j, k)) - ap * (q_ext(q, g, i + 1, j, k) - qp) +
           alpha[p - n] * (qp - q_ext(q, g, i, j - 1, k)) - ap * (q_ext(q, g, i, j + 1, k) - qp);
  if (DIM == 3) {
    const int64_t n2 = n * n;
    s += alpha[p - n2] * (qp - q_ext(q, g, i, j, k - 1)) - ap * (q_ext(q, g, i, j, k + 1) - qp);
    return Real(2) * Real(1.0 / g.ne) * s;
  }
  return Real(2) * s;
}

}  // namespace crv
