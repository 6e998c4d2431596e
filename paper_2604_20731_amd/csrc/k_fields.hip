// Field kernels of the coupled step: coefficient refresh (alpha), collocation
// residual, adjoint of the robust loss, pressure projection, explicit
// saturation assembly, and the float64 factorisations done once at init.
//
// Layouts: nodal arrays (N+1)^d with x fastest; interior arrays padded to a
// pitch mp per row, row index j-1 (2D); coefficient arrays nb^d.
#include "kernels.h"
#include "stencil.h"

namespace crv {

// ---------------------------------------------------------------------------
// a1: S at the nodes and alpha = K (kr_w/mu_w + kr_g/mu_g)   (second eq. 23)
// ---------------------------------------------------------------------------
template <typename Real, int R>
__global__ __launch_bounds__(256) void k_refresh2(Geom g, const Real* __restrict__ c,
                                                  const int* __restrict__ kf,
                                                  const Real* __restrict__ kv,
                                                  const Real* __restrict__ perm, Real inv_mu_w,
                                                  Real inv_mu_g, Real nexp, Real rw_mu, Real rg_mu,
                                                  Real* __restrict__ s_nodal,
                                                  Real* __restrict__ alpha,
                                                  Real* __restrict__ flux, int64_t zb) {
  c = zofs(c, zb); kf = zofs(kf, zb); kv = zofs(kv, zb); perm = zofs(perm, zb);
  s_nodal = zofs(s_nodal, zb); alpha = zofs(alpha, zb); flux = zofs(flux, zb);
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int n = g.n;
  if (p >= int64_t(n) * n) return;
  const int i = int(p % n), j = int(p / n);
  const int fi = kf[i], fj = kf[j];
  Real s = 0;
#pragma unroll
  for (int b = 0; b <= R; ++b) {
    Real row = 0;
#pragma unroll
    for (int a = 0; a <= R; ++a) row += kv[i * (R + 1) + a] * c[int64_t(fj + b) * g.nb + fi + a];
    s += kv[j * (R + 1) + b] * row;
  }
  const Real sc = clamp01(s);
  const Real krw = powi_or_pow(Real(1) - sc, nexp), krg = powi_or_pow(sc, nexp);
  s_nodal[p] = s;
  alpha[p] = (krw * inv_mu_w + krg * inv_mu_g) * perm[p];
  if (flux) flux[p] = (krw * rw_mu + krg * rg_mu) * perm[p];
}

template <typename Real, int R>
__global__ __launch_bounds__(256) void k_refresh3(Geom g, const Real* __restrict__ c,
                                                  const int* __restrict__ kf,
                                                  const Real* __restrict__ kv,
                                                  const Real* __restrict__ perm, Real inv_mu_w,
                                                  Real inv_mu_g, Real nexp, Real rw_mu, Real rg_mu,
                                                  Real* __restrict__ s_nodal,
                                                  Real* __restrict__ alpha,
                                                  Real* __restrict__ flux) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int n = g.n, nb = g.nb;
  if (p >= int64_t(n) * n * n) return;
  const int i = int(p % n), j = int((p / n) % n), k = int(p / (int64_t(n) * n));
  const int fi = kf[i], fj = kf[j], fk = kf[k];
  Real s = 0;
#pragma unroll
  for (int cc = 0; cc <= R; ++cc) {
    Real plane = 0;
#pragma unroll
    for (int b = 0; b <= R; ++b) {
      Real row = 0;
#pragma unroll
      for (int a = 0; a <= R; ++a)
        row += kv[i * (R + 1) + a] * c[(int64_t(fk + cc) * nb + fj + b) * nb + fi + a];
      plane += kv[j * (R + 1) + b] * row;
    }
    s += kv[k * (R + 1) + cc] * plane;
  }
  const Real sc = clamp01(s);
  const Real krw = powi_or_pow(Real(1) - sc, nexp), krg = powi_or_pow(sc, nexp);
  s_nodal[p] = s;
  alpha[p] = (krw * inv_mu_w + krg * inv_mu_g) * perm[p];
  if (flux) flux[p] = (krw * rw_mu + krg * rg_mu) * perm[p];
}

template <typename Real>
void launch_refresh(const Geom& g, const Real* s_coefs, const int* kf, const Real* kv,
                    const Real* perm, double mu_w, double mu_g, double nexp, double rho_w,
                    double rho_g, Real* s_nodal, Real* alpha, Real* flux, hipStream_t st,
                    Batch bz) {
  const Real iw = Real(1.0 / mu_w), ig = Real(1.0 / mu_g), ne = Real(nexp);
  const Real rw = Real(rho_w / mu_w), rg = Real(rho_g / mu_g);
  if (g.dim == 3) {
    dim3 grid3(cdiv(ipow(g.n, 3), 256));
    switch (g.r) {
      case 1: k_refresh3<Real, 1><<<grid3, 256, 0, st>>>(g, s_coefs, kf, kv, perm, iw, ig, ne, rw, rg, s_nodal, alpha, flux); break;
      case 2: k_refresh3<Real, 2><<<grid3, 256, 0, st>>>(g, s_coefs, kf, kv, perm, iw, ig, ne, rw, rg, s_nodal, alpha, flux); break;
      default: k_refresh3<Real, 3><<<grid3, 256, 0, st>>>(g, s_coefs, kf, kv, perm, iw, ig, ne, rw, rg, s_nodal, alpha, flux); break;
    }
    return;
  }
  const int64_t tot = int64_t(g.n) * g.n;
  dim3 grid(cdiv(tot, 256), 1, bz.n);
  switch (g.r) {
    case 1: k_refresh2<Real, 1><<<grid, 256, 0, st>>>(g, s_coefs, kf, kv, perm, iw, ig, ne, rw, rg, s_nodal, alpha, flux, bz.zb); break;
    case 2: k_refresh2<Real, 2><<<grid, 256, 0, st>>>(g, s_coefs, kf, kv, perm, iw, ig, ne, rw, rg, s_nodal, alpha, flux, bz.zb); break;
    default: k_refresh2<Real, 3><<<grid, 256, 0, st>>>(g, s_coefs, kf, kv, perm, iw, ig, ne, rw, rg, s_nodal, alpha, flux, bz.zb); break;
  }
}

// Pressure right-hand side with gravity: h^d (q - div_+(g F)) with g = -gravity
// e_v (e_v: y in 2D, z in 3D) and F the buoyancy flux from the refresh, i.e.
// hq_p = h^d q_p + gravity h^(d-1) (F_{p+e_v} - F_p) (the RHS_ij formula of
// the CRVPINN section; forward difference, eq. 22).  Top-face nodes, which no
// interior residual reads, keep h^d q.
template <typename Real>
__global__ __launch_bounds__(256) void k_gravity_rhs(int64_t total, int64_t sv, int64_t top,
                                                     const Real* __restrict__ flux,
                                                     const Real* __restrict__ qi,
                                                     const Real* __restrict__ qp, Real hd,
                                                     Real gh, Real* __restrict__ hq, int64_t zb) {
  flux = zofs(flux, zb); qi = zofs(qi, zb); qp = zofs(qp, zb); hq = zofs(hq, zb);
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= total) return;
  Real v = hd * (qi[p] + qp[p]);
  if (p < top) v += gh * (flux[p + sv] - flux[p]);
  hq[p] = v;
}

template <typename Real>
void launch_gravity_rhs(const Geom& g, const Real* flux, const Real* qi, const Real* qp,
                        double gravity, Real* hq, hipStream_t st, Batch bz) {
  const int64_t n = g.n, total = ipow(g.n, g.dim);
  const int64_t sv = g.dim == 3 ? n * n : n;  // stride of the vertical axis
  const double h = 1.0 / g.ne;
  k_gravity_rhs<Real><<<dim3(cdiv(total, 256), 1, bz.n), 256, 0, st>>>(
      total, sv, total - sv, flux, qi, qp, Real(std::pow(h, g.dim)),
      Real(gravity * std::pow(h, g.dim - 1)), hq, bz.zb);
}

// ---------------------------------------------------------------------------
// a3: RES_p = sum_dir [alpha_{p-e}(u_p - u_{p-e}) - alpha_p (u_{p+e} - u_p)] - h^2 q_p
// (eq. 24-25 with Kronecker-delta tests at interior nodes)
// ---------------------------------------------------------------------------
// 2D: 64 x 16 tiles of interior nodes.  The block stages u over the tile and
// its one-node halo, and alpha over the tile and its lower/left neighbours, in
// LDS with coalesced row loads (each value read from memory once per tile),
// then each thread forms four outputs of its column from LDS.
constexpr int RTX = 64, RTY = 16;
template <typename Real>
__global__ __launch_bounds__(256) void k_residual2(Geom g, const Real* __restrict__ u,
                                                   const Real* __restrict__ alpha,
                                                   const Real* __restrict__ hq,
                                                   Real* __restrict__ res, int64_t zb) {
  u = zofs(u, zb); alpha = zofs(alpha, zb); hq = zofs(hq, zb); res = zofs(res, zb);
  __shared__ Real su[RTY + 2][RTX + 2];  // node rows j0 .. j0 + RTY + 1, cols i0 .. i0 + RTX + 1
  __shared__ Real sa[RTY + 1][RTX + 1];  // node rows j0 .. j0 + RTY, cols i0 .. i0 + RTX
  const int n = g.n;
  const int i0 = blockIdx.x * RTX, j0 = blockIdx.y * RTY;  // first interior column / row (node - 1)
  const int lx = threadIdx.x & 63, ii = i0 + lx;
  // every load of the thread is issued before the first wait: h^2 q of its
  // outputs, then its share of the two tiles
  Real hv[RTY / 4];
#pragma unroll
  for (int k = 0; k < RTY / 4; ++k) {
    const int jj = j0 + (threadIdx.x >> 6) + 4 * k;
    hv[k] = (ii < g.m && jj < g.m) ? hq[int64_t(jj + 1) * n + (ii + 1)] : Real(0);
  }
  constexpr int NU = (RTY + 2) * (RTX + 2), NA = (RTY + 1) * (RTX + 1);
  constexpr int IU = (NU + 255) / 256, IA = (NA + 255) / 256;
  // the tile values go to registers first and to LDS afterwards, so that no
  // LDS store sits between two loads and waits for the earlier one
  Real ru[IU], ra[IA];
#pragma unroll
  for (int it = 0; it < IU; ++it) {
    const int k = threadIdx.x + 256 * it;
    const int r = k / (RTX + 2), c = k - r * (RTX + 2);
    const int nr = j0 + r, nc = i0 + c;
    ru[it] = (k < NU && nr < n && nc < n) ? u[int64_t(nr) * n + nc] : Real(0);
  }
#pragma unroll
  for (int it = 0; it < IA; ++it) {
    const int k = threadIdx.x + 256 * it;
    const int r = k / (RTX + 1), c = k - r * (RTX + 1);
    const int nr = j0 + r, nc = i0 + c;
    ra[it] = (k < NA && nr < n && nc < n) ? alpha[int64_t(nr) * n + nc] : Real(0);
  }
#pragma unroll
  for (int it = 0; it < IU; ++it) {
    const int k = threadIdx.x + 256 * it;
    const int r = k / (RTX + 2), c = k - r * (RTX + 2);
    if (k < NU) su[r][c] = ru[it];
  }
#pragma unroll
  for (int it = 0; it < IA; ++it) {
    const int k = threadIdx.x + 256 * it;
    const int r = k / (RTX + 1), c = k - r * (RTX + 1);
    if (k < NA) sa[r][c] = ra[it];
  }
  __syncthreads();
  if (ii >= g.m) return;
#pragma unroll
  for (int k = 0; k < RTY / 4; ++k) {
    const int ly = (threadIdx.x >> 6) + 4 * k, jj = j0 + ly;
    if (jj >= g.m) break;
    const Real up = su[ly + 1][lx + 1], ap = sa[ly + 1][lx + 1];
    const Real r = sa[ly + 1][lx] * (up - su[ly + 1][lx]) - ap * (su[ly + 1][lx + 2] - up) +
                   sa[ly][lx + 1] * (up - su[ly][lx + 1]) - ap * (su[ly + 2][lx + 1] - up) - hv[k];
    res[int64_t(jj) * g.mp + ii] = r;
  }
}

// 3D: RES_p = h sum_dir [...] - h^3 q_p (the alpha terms carry h^(d-2));
// interior arrays padded to mp in every direction
template <typename Real>
__global__ __launch_bounds__(256) void k_residual3(Geom g, const Real* __restrict__ u,
                                                   const Real* __restrict__ alpha,
                                                   const Real* __restrict__ hq, Real h,
                                                   Real* __restrict__ res) {
  const int ii = blockIdx.x * 64 + (threadIdx.x & 63);
  const int jj = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int kk = blockIdx.z;
  if (ii >= g.m || jj >= g.m) return;
  const int64_t n = g.n, n2 = n * n;
  const int64_t p = (int64_t(kk + 1) * n + (jj + 1)) * n + (ii + 1);
  const Real up = u[p], ap = alpha[p];
  const Real sx = alpha[p - 1] * (up - u[p - 1]) - ap * (u[p + 1] - up);
  const Real sy = alpha[p - n] * (up - u[p - n]) - ap * (u[p + n] - up);
  const Real sz = alpha[p - n2] * (up - u[p - n2]) - ap * (u[p + n2] - up);
  res[(int64_t(kk) * g.mp + jj) * g.mp + ii] = h * (sx + sy + sz) - hq[p];
}

template <typename Real>
void launch_residual(const Geom& g, const Real* u, const Real* alpha, const Real* hq, Real* res,
                     hipStream_t st, Batch bz) {
  if (g.dim == 3) {
    dim3 grid3(cdiv(g.m, 64), cdiv(g.m, 4), g.m);
    k_residual3<Real><<<grid3, 256, 0, st>>>(g, u, alpha, hq, Real(1.0 / g.ne), res);
    return;
  }
  dim3 grid(cdiv(g.m, RTX), cdiv(g.m, RTY), bz.n);
  k_residual2<Real><<<grid, 256, 0, st>>>(g, u, alpha, hq, res, bz.zb);
}

// ---------------------------------------------------------------------------
// a5: g_u = 2 A^T q~ on the full grid (q~ = q inside, 0 on the boundary; the
// boundary entries are zero because the trial functions vanish there), and
// per-block partial sums of LOSS = RES . q (eq. 27).  With observations
// (obs_w non-null) the data misfit w (u - d)^2 of the inverse problem joins
// the loss and 2 w (u - d) joins g_u at interior nodes.
// ---------------------------------------------------------------------------
template <typename Real, int DIM>
__global__ __launch_bounds__(256) void k_adjoint(Geom g, const Real* __restrict__ q,
                                                 const Real* __restrict__ alpha,
                                                 const Real* __restrict__ res,
                                                 Real* __restrict__ gu,
                                                 Real* __restrict__ partials,
                                                 const Real* __restrict__ obs_w,
                                                 const Real* __restrict__ obs_d,
                                                 const Real* __restrict__ u) {
  __shared__ Real sbuf[256];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  const int n = g.n;
  Real lpart = 0;
  if (i < n && j < n) {
    const int64_t p = (int64_t(k) * n + j) * n + i;
    int64_t iq;
    Real gv = adjoint_at<Real, DIM>(g, q, alpha, p, &iq);
    if (iq >= 0) {
      lpart = res[iq] * q[iq];
      if (obs_w) {
        const Real w = obs_w[p], r = u[p] - obs_d[p];
        gv += Real(2) * w * r;
        lpart += w * r * r;
      }
    }
    gu[p] = gv;
  }
  const Real tot = block_sum(lpart, sbuf);
  if (threadIdx.x == 0) partials[(int64_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
}

int adjoint_partials(const Geom& g) {
  return cdiv(g.n, 64) * cdiv(g.n, 4) * (g.dim == 3 ? g.n : 1);
}

template <typename Real>
int launch_adjoint(const Geom& g, const Real* q, const Real* alpha, const Real* res, Real* gu,
                   Real* partials, hipStream_t st, const Real* obs_w, const Real* obs_d,
                   const Real* u) {
  if (g.dim == 3) {
    dim3 grid3(cdiv(g.n, 64), cdiv(g.n, 4), g.n);
    k_adjoint<Real, 3><<<grid3, 256, 0, st>>>(g, q, alpha, res, gu, partials, obs_w, obs_d, u);
    return grid3.x * grid3.y * grid3.z;
  }
  dim3 grid(cdiv(g.n, 64), cdiv(g.n, 4));
  k_adjoint<Real, 2><<<grid, 256, 0, st>>>(g, q, alpha, res, gu, partials, obs_w, obs_d, u);
  return grid.x * grid.y;
}

// Adam on the nodal log K of the inverse problem (its own moments; step
// count *t, advanced before the launch), then K = exp(log K)
template <typename Real>
__global__ __launch_bounds__(256) void k_adam_logk(int64_t n, Real* __restrict__ logk,
                                                   Real* __restrict__ m, Real* __restrict__ v,
                                                   const Real* __restrict__ g,
                                                   Real* __restrict__ perm, double lr, double b1,
                                                   double b2, double eps,
                                                   const long long* __restrict__ t) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double tt = double(*t);
  const Real c1 = Real(1.0 - pow(b1, tt)), c2 = Real(1.0 - pow(b2, tt));
  const Real gg = g[p];
  const Real mm = Real(b1) * m[p] + Real(1.0 - b1) * gg;
  const Real vv = Real(b2) * v[p] + Real(1.0 - b2) * gg * gg;
  m[p] = mm;
  v[p] = vv;
  const Real nl = logk[p] - Real(lr) * (mm / c1) / (sqrt(vv / c2) + Real(eps));
  logk[p] = nl;
  perm[p] = exp(nl);
}

template <typename Real>
void launch_adam_logk(int64_t n, Real* logk, Real* m, Real* v, const Real* g, Real* perm,
                      double lr, double b1, double b2, double eps, const long long* t,
                      hipStream_t st) {
  k_adam_logk<Real><<<cdiv(n, 256), 256, 0, st>>>(n, logk, m, v, g, perm, lr, b1, b2, eps, t);
}

// log K taken from a device array: log K copied, K = exp(log K) evaluated in
// float64 and rounded once, as the host path does
__global__ __launch_bounds__(256) void k_set_logk(int64_t n, const float* __restrict__ src,
                                                  float* __restrict__ logk,
                                                  float* __restrict__ perm) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float lk = src[p];
  logk[p] = lk;
  perm[p] = float(exp(double(lk)));
}

void launch_set_logk(int64_t n, const float* src, float* logk, float* perm, hipStream_t st) {
  if (n == 0) return;
  k_set_logk<<<cdiv(n, 256), 256, 0, st>>>(n, src, logk, perm);
}

template <typename Real>
__global__ __launch_bounds__(256) void k_loss_finalize(const Real* __restrict__ part, int np,
                                                       double* __restrict__ hist, int cap,
                                                       const long long* __restrict__ t_dev,
                                                       int slot_offset) {
  __shared__ double sbuf[256];
  double v = 0;
  for (int k = threadIdx.x; k < np; k += 256) v += double(part[k]);
  const double tot = block_sum(v, sbuf);
  if (threadIdx.x == 0) hist[(*t_dev + slot_offset) % cap] = tot;
}

template <typename Real>
void launch_loss_finalize(const Real* partials, int np, double* loss_hist, int cap,
                          const long long* t_dev, int slot_offset, hipStream_t st) {
  k_loss_finalize<Real><<<1, 256, 0, st>>>(partials, np, loss_hist, cap, t_dev, slot_offset);
}

// dLOSS/dalpha_p = 2 sum_dir (u_{p+e}-u_p)(q_{p+e}-q_p) (2D, q zero-extended);
// dLOSS/dlogK = dLOSS/dalpha * alpha.  With gravity the right-hand side holds
// h^d div_+(g F) with F linear in K, which adds
// -2 gravity h^(d-1) F_p (q_{p-e_v} - q_p) (gf = 2 gravity h^(d-1); flux null
// without gravity).
template <typename Real>
__global__ __launch_bounds__(256) void k_grad_logperm2(Geom g, const Real* __restrict__ u,
                                                       const Real* __restrict__ q,
                                                       const Real* __restrict__ alpha,
                                                       const Real* __restrict__ flux, Real gf,
                                                       Real* __restrict__ out) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int n = g.n;
  if (i >= n || j >= n) return;
  const int64_t p = int64_t(j) * n + i;
  const Real qp = q_ext(q, g, i, j, 1);
  Real s = 0;
  if (i + 1 < n) s += (u[p + 1] - u[p]) * (q_ext(q, g, i + 1, j, 1) - qp);
  if (j + 1 < n) s += (u[p + n] - u[p]) * (q_ext(q, g, i, j + 1, 1) - qp);
  Real r = Real(2) * s * alpha[p];
  if (flux) r -= gf * flux[p] * (q_ext(q, g, i, j - 1, 1) - qp);
  out[p] = r;
}

template <typename Real>
__global__ __launch_bounds__(256) void k_grad_logperm3(Geom g, const Real* __restrict__ u,
                                                       const Real* __restrict__ q,
                                                       const Real* __restrict__ alpha, Real h,
                                                       const Real* __restrict__ flux, Real gf,
                                                       Real* __restrict__ out) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  const int64_t n = g.n, n2 = n * n;
  if (i >= n || j >= n) return;
  const int64_t p = (int64_t(k) * n + j) * n + i;
  const Real qp = q_ext(q, g, i, j, k);
  Real s = 0;
  if (i + 1 < n) s += (u[p + 1] - u[p]) * (q_ext(q, g, i + 1, j, k) - qp);
  if (j + 1 < n) s += (u[p + n] - u[p]) * (q_ext(q, g, i, j + 1, k) - qp);
  if (k + 1 < n) s += (u[p + n2] - u[p]) * (q_ext(q, g, i, j, k + 1) - qp);
  Real r = Real(2) * h * s * alpha[p];
  if (flux) r -= gf * flux[p] * (q_ext(q, g, i, j, k - 1) - qp);
  out[p] = r;
}

template <typename Real>
void launch_grad_logperm(const Geom& g, const Real* u, const Real* q, const Real* alpha,
                         const Real* flux, double gravity, Real* out, hipStream_t st) {
  const Real gf = Real(2.0 * gravity * std::pow(1.0 / g.ne, g.dim - 1));
  if (g.dim == 3) {
    dim3 grid3(cdiv(g.n, 64), cdiv(g.n, 4), g.n);
    k_grad_logperm3<Real><<<grid3, 256, 0, st>>>(g, u, q, alpha, Real(1.0 / g.ne), flux, gf, out);
    return;
  }
  dim3 grid(cdiv(g.n, 64), cdiv(g.n, 4));
  k_grad_logperm2<Real><<<grid, 256, 0, st>>>(g, u, q, alpha, flux, gf, out);
}

// ---------------------------------------------------------------------------
// a8: b_kl = sum_ij Q_l(j) Q_k(i) u_ij with Q_k(i) = int B_k hat_i (algorithm step 4)
// ---------------------------------------------------------------------------
template <typename Real, int R>
__global__ __launch_bounds__(256) void k_project2(Geom g, const Real* __restrict__ u,
                                                  const Real* __restrict__ qv,
                                                  Real* __restrict__ b, int64_t zb) {
  u = zofs(u, zb); qv = zofs(qv, zb); b = zofs(b, zb);
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int nb = g.nb;
  if (idx >= int64_t(nb) * nb) return;
  const int k = int(idx % nb), l = int(idx / nb);
  Real acc = 0;
#pragma unroll
  for (int tb = 0; tb < R + 2; ++tb) {
    const int j = l - R + tb;
    if (j < 0 || j > g.ne) continue;
    Real row = 0;
#pragma unroll
    for (int ta = 0; ta < R + 2; ++ta) {
      const int i = k - R + ta;
      if (i < 0 || i > g.ne) continue;
      row += qv[k * (R + 2) + ta] * u[int64_t(j) * g.n + i];
    }
    acc += qv[l * (R + 2) + tb] * row;
  }
  b[idx] = acc;
}

template <typename Real, int R>
__global__ __launch_bounds__(256) void k_project3(Geom g, const Real* __restrict__ u,
                                                  const Real* __restrict__ qv,
                                                  Real* __restrict__ b) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int nb = g.nb, n = g.n;
  if (idx >= int64_t(nb) * nb * nb) return;
  const int a = int(idx % nb), bb = int((idx / nb) % nb), c = int(idx / (int64_t(nb) * nb));
  Real acc = 0;
#pragma unroll
  for (int tc = 0; tc < R + 2; ++tc) {
    const int k = c - R + tc;
    if (k < 0 || k > g.ne) continue;
    Real plane = 0;
#pragma unroll
    for (int tb = 0; tb < R + 2; ++tb) {
      const int j = bb - R + tb;
      if (j < 0 || j > g.ne) continue;
      Real row = 0;
#pragma unroll
      for (int ta = 0; ta < R + 2; ++ta) {
        const int i = a - R + ta;
        if (i < 0 || i > g.ne) continue;
        row += qv[a * (R + 2) + ta] * u[(int64_t(k) * n + j) * n + i];
      }
      plane += qv[bb * (R + 2) + tb] * row;
    }
    acc += qv[c * (R + 2) + tc] * plane;
  }
  b[idx] = acc;
}

template <typename Real>
void launch_project(const Geom& g, const Real* u, const Real* qv, Real* b, hipStream_t st,
                    Batch bz) {
  if (g.dim == 3) {
    dim3 grid3(cdiv(ipow(g.nb, 3), 256));
    switch (g.r) {
      case 1: k_project3<Real, 1><<<grid3, 256, 0, st>>>(g, u, qv, b); break;
      case 2: k_project3<Real, 2><<<grid3, 256, 0, st>>>(g, u, qv, b); break;
      default: k_project3<Real, 3><<<grid3, 256, 0, st>>>(g, u, qv, b); break;
    }
    return;
  }
  dim3 grid(cdiv(int64_t(g.nb) * g.nb, 256), 1, bz.n);
  switch (g.r) {
    case 1: k_project2<Real, 1><<<grid, 256, 0, st>>>(g, u, qv, b, bz.zb); break;
    case 2: k_project2<Real, 2><<<grid, 256, 0, st>>>(g, u, qv, b, bz.zb); break;
    default: k_project2<Real, 3><<<grid, 256, 0, st>>>(g, u, qv, b, bz.zb); break;
  }
}

// ---------------------------------------------------------------------------
// a10: explicit saturation right-hand side (eq. 10, Galerkin form eq. 12),
// owner-computes tiles: a block owns TC x TC coefficients, evaluates the
// integrand at the Gauss points of every element touching them into LDS, and
// gathers its coefficients' sums in a fixed order (no atomics).
// ---------------------------------------------------------------------------
template <typename Real, int R, int TC>
__global__ __launch_bounds__(TC* TC) void k_ads_assemble2(
    Geom g, const Real* __restrict__ sc, const Real* __restrict__ pc,
    const Real* __restrict__ perm, const Real* __restrict__ poro, const Real* __restrict__ qi,
    const Real* __restrict__ qp, const Real* __restrict__ gb, const Real* __restrict__ gdb,
    const Real* __restrict__ gxi, const Real* __restrict__ gw, const double* __restrict__ tau_dev,
    Real inv_mu_w, Real inv_mu_g, Real nexp, Real gshift, Real* __restrict__ b, int64_t zb) {
  sc = zofs(sc, zb); pc = zofs(pc, zb); perm = zofs(perm, zb); poro = zofs(poro, zb);
  qi = zofs(qi, zb); qp = zofs(qp, zb); gb = zofs(gb, zb); gdb = zofs(gdb, zb);
  gxi = zofs(gxi, zb); gw = zofs(gw, zb); tau_dev = zofs(tau_dev, zb); b = zofs(b, zb);
  const Real tau = Real(*tau_dev);
  constexpr int NG = R + 1;          // Gauss points per element and axis
  constexpr int TE = TC + R;         // elements per tile and axis
  constexpr int TCO = TC + 2 * R;    // coefficients touched per axis
  constexpr int TN = TE + 1;         // nodes per axis
  constexpr int GP = TE * NG;        // Gauss points per axis
  __shared__ Real sS[TCO * TCO], sP[TCO * TCO];
  __shared__ Real sK[TN * TN], sF[TN * TN], sQi[TN * TN], sQp[TN * TN];
  __shared__ Real sF0[GP * GP], sFx[GP * GP], sFy[GP * GP];
  const int tid = threadIdx.x;
  const int k0 = blockIdx.x * TC, l0 = blockIdx.y * TC;
  const int c0x = k0 - R, c0y = l0 - R;  // first touched coefficient / element / node
  const int nb = g.nb, ne = g.ne, n = g.n;
  // the tile's values go to registers first and to LDS afterwards, so that
  // no LDS store sits between two loads and waits for the earlier one
  constexpr int NT = TC * TC, IC = (TCO * TCO + NT - 1) / NT, IN = (TN * TN + NT - 1) / NT;
  Real rS[IC], rP[IC], rK[IN], rF[IN], rQi[IN], rQp[IN];
#pragma unroll
  for (int it = 0; it < IC; ++it) {
    const int t = tid + NT * it;
    const int a = c0x + t % TCO, bb = c0y + t / TCO;
    const bool ok = t < TCO * TCO && a >= 0 && a < nb && bb >= 0 && bb < nb;
    rS[it] = ok ? sc[int64_t(bb) * nb + a] : Real(0);
    rP[it] = ok ? pc[int64_t(bb) * nb + a] : Real(0);
  }
#pragma unroll
  for (int it = 0; it < IN; ++it) {
    const int t = tid + NT * it;
    const int i = c0x + t % TN, j = c0y + t / TN;
    const bool ok = t < TN * TN && i >= 0 && i <= ne && j >= 0 && j <= ne;
    const int64_t p = int64_t(j) * n + i;
    rK[it] = ok ? perm[p] : Real(0);
    rF[it] = ok ? poro[p] : Real(1);
    rQi[it] = ok ? qi[p] : Real(0);
    rQp[it] = ok ? qp[p] : Real(0);
  }
#pragma unroll
  for (int it = 0; it < IC; ++it) {
    const int t = tid + NT * it;
    if (t < TCO * TCO) {
      sS[t] = rS[it];
      sP[t] = rP[it];
    }
  }
#pragma unroll
  for (int it = 0; it < IN; ++it) {
    const int t = tid + NT * it;
    if (t < TN * TN) {
      sK[t] = rK[it];
      sF[t] = rF[it];
      sQi[t] = rQi[it];
      sQp[t] = rQp[it];
    }
  }
  __syncthreads();
  for (int t = tid; t < GP * GP; t += TC * TC) {
    const int gxl = t % GP, gyl = t / GP;
    const int exl = gxl / NG, gx = gxl % NG, eyl = gyl / NG, gy = gyl % NG;
    const int ex = c0x + exl, ey = c0y + eyl;
    Real f0 = 0, fx = 0, fy = 0;
    if (ex >= 0 && ex < ne && ey >= 0 && ey < ne) {
      const Real* bx = gb + (int64_t(ex) * NG + gx) * (R + 1);
      const Real* dbx = gdb + (int64_t(ex) * NG + gx) * (R + 1);
      const Real* by = gb + (int64_t(ey) * NG + gy) * (R + 1);
      const Real* dby = gdb + (int64_t(ey) * NG + gy) * (R + 1);
      Real s = 0, px = 0, py = 0;
#pragma unroll
      for (int bb = 0; bb <= R; ++bb) {
        Real rs = 0, rp = 0, rdp = 0;
#pragma unroll
        for (int a = 0; a <= R; ++a) {
          const int li = (eyl + bb) * TCO + exl + a;
          rs += bx[a] * sS[li];
          rp += dbx[a] * sP[li];
          rdp += bx[a] * sP[li];
        }
        s += by[bb] * rs;
        px += by[bb] * rp;
        py += dby[bb] * rdp;
      }
      // Q1 interpolation of the nodal data at the Gauss point
      const Real xi = gxi[gx], eta = gxi[gy];
      const Real w00 = (1 - xi) * (1 - eta), w10 = xi * (1 - eta), w01 = (1 - xi) * eta, w11 = xi * eta;
      const int n00 = eyl * TN + exl;
      auto interp = [&](const Real* a) {
        return w00 * a[n00] + w10 * a[n00 + 1] + w01 * a[n00 + TN] + w11 * a[n00 + TN + 1];
      };
      const Real kk = interp(sK), phi = interp(sF), qin = interp(sQi), qpr = interp(sQp);
      const Real scl = clamp01(s);
      const Real lam_g = powi_or_pow(scl, nexp) * inv_mu_g;
      const Real lam_w = powi_or_pow(Real(1) - scl, nexp) * inv_mu_w;
      const Real fg = lam_g / (lam_g + lam_w);
      const Real qg = qin + fg * qpr;
      const Real w = gw[gx] * gw[gy];
      const Real tphi = tau / phi;
      f0 = w * (s + tphi * qg);
      const Real c = -w * tphi * lam_g * kk;
      fx = c * px;
      fy = c * (py + gshift);  // grad p - rho_g g, g = -gravity e_y
    }
    sF0[t] = f0;
    sFx[t] = fx;
    sFy[t] = fy;
  }
  __syncthreads();
  const int tx = tid % TC, ty = tid / TC;
  const int k = k0 + tx, l = l0 + ty;
  if (k >= nb || l >= nb) return;
  Real acc = 0;
  for (int ey = l - R; ey <= l; ++ey) {
    if (ey < 0 || ey >= ne) continue;
    const int bb = l - ey, eyl = ey - c0y;
    for (int ex = k - R; ex <= k; ++ex) {
      if (ex < 0 || ex >= ne) continue;
      const int a = k - ex, exl = ex - c0x;
#pragma unroll
      for (int gy = 0; gy < NG; ++gy) {
        const Real by = gb[(int64_t(ey) * NG + gy) * (R + 1) + bb];
        const Real dby = gdb[(int64_t(ey) * NG + gy) * (R + 1) + bb];
        Real rx0 = 0, rxx = 0, rxy = 0;
#pragma unroll
        for (int gx = 0; gx < NG; ++gx) {
          const Real bx = gb[(int64_t(ex) * NG + gx) * (R + 1) + a];
          const Real dbx = gdb[(int64_t(ex) * NG + gx) * (R + 1) + a];
          const int t = (eyl * NG + gy) * GP + exl * NG + gx;
          rx0 += bx * sF0[t];
          rxx += dbx * sFx[t];
          rxy += bx * sFy[t];
        }
        acc += by * (rx0 + rxx) + dby * rxy;
      }
    }
  }
  b[int64_t(l) * nb + k] = acc;
}

// 3D form: a block owns TC x TC coefficients in (x, y) and ZC consecutive
// coefficients in z, and streams through the element layers that touch them.
// Per layer: integrand at the Gauss points of the (TC+R)^2 elements of the
// layer (LDS), contraction with the x test functions, then with the y test
// functions (sum factorisation), then each owning thread adds the z test
// functions into R+1 rolling accumulators; coefficient c is complete once
// layer c has been added.  Fixed order throughout, no atomics.
template <typename Real, int R, int TC, int ZC>
__global__ __launch_bounds__(256) void k_ads_assemble3(
    Geom g, const Real* __restrict__ sc, const Real* __restrict__ pc,
    const Real* __restrict__ perm, const Real* __restrict__ poro, const Real* __restrict__ qi,
    const Real* __restrict__ qp, const Real* __restrict__ gb, const Real* __restrict__ gdb,
    const Real* __restrict__ gxi, const Real* __restrict__ gw, const double* __restrict__ tau_dev,
    Real inv_mu_w, Real inv_mu_g, Real nexp, Real gshift, Real* __restrict__ b) {
  constexpr int NG = R + 1;
  constexpr int TE = TC + R;
  constexpr int TCO = TC + 2 * R;
  constexpr int TN = TE + 1;
  constexpr int GP = TE * NG;
  constexpr int NT = 256;
  static_assert(sizeof(Real) * (2 * TCO * TCO * (R + 1) + 8 * TN * TN + 4 * GP * GP * NG +
                                3 * TC * GP * NG + 2 * TC * TC * NG) <= 65536,
                "LDS of the 3D assembly tile");
  __shared__ Real sS[(R + 1) * TCO * TCO], sP[(R + 1) * TCO * TCO];
  __shared__ Real sK[2 * TN * TN], sF[2 * TN * TN], sQi[2 * TN * TN], sQp[2 * TN * TN];
  __shared__ Real sF0[GP * GP * NG], sFx[GP * GP * NG], sFy[GP * GP * NG], sFz[GP * GP * NG];
  __shared__ Real sG0[TC * GP * NG], sGy[TC * GP * NG], sGz[TC * GP * NG];
  __shared__ Real sH0[TC * TC * NG], sHz[TC * TC * NG];
  const Real tau = Real(*tau_dev);
  const int tid = threadIdx.x;
  const int k0 = blockIdx.x * TC, l0 = blockIdx.y * TC, cz0 = blockIdx.z * ZC;
  const int c0x = k0 - R, c0y = l0 - R;
  const int nb = g.nb, ne = g.ne;
  const int64_t n = g.n, nbb = int64_t(nb) * nb;
  const int own_a = tid % TC, own_b = tid / TC;
  const bool owner = tid < TC * TC;
  const int kx = k0 + own_a, ly = l0 + own_b;
  Real acc[R + 1];
#pragma unroll
  for (int j = 0; j <= R; ++j) acc[j] = 0;
  const int ez_end = min(cz0 + ZC, nb);
  for (int ez = cz0 - R; ez < ez_end; ++ez) {
    if (ez >= 0 && ez < ne) {
      // coefficient planes ez..ez+R and nodal planes ez, ez+1 of the tile
      for (int t = tid; t < (R + 1) * TCO * TCO; t += NT) {
        const int a = c0x + t % TCO, bb = c0y + (t / TCO) % TCO, cc = ez + t / (TCO * TCO);
        const bool ok = a >= 0 && a < nb && bb >= 0 && bb < nb;
        const int64_t q = int64_t(cc) * nbb + int64_t(bb) * nb + a;
        sS[t] = ok ? sc[q] : Real(0);
        sP[t] = ok ? pc[q] : Real(0);
      }
      for (int t = tid; t < 2 * TN * TN; t += NT) {
        const int i = c0x + t % TN, j = c0y + (t / TN) % TN, k = ez + t / (TN * TN);
        const bool ok = i >= 0 && i <= ne && j >= 0 && j <= ne;
        const int64_t q = (int64_t(k) * n + j) * n + i;
        sK[t] = ok ? perm[q] : Real(0);
        sF[t] = ok ? poro[q] : Real(1);
        sQi[t] = ok ? qi[q] : Real(0);
        sQp[t] = ok ? qp[q] : Real(0);
      }
      __syncthreads();
      // integrand at the Gauss points of the layer
      for (int t = tid; t < GP * GP * NG; t += NT) {
        const int gxl = t % GP, gyl = (t / GP) % GP, gz = t / (GP * GP);
        const int exl = gxl / NG, gx = gxl % NG, eyl = gyl / NG, gy = gyl % NG;
        const int ex = c0x + exl, ey = c0y + eyl;
        Real f0 = 0, fx = 0, fy = 0, fz = 0;
        if (ex >= 0 && ex < ne && ey >= 0 && ey < ne) {
          const Real* bx = gb + (int64_t(ex) * NG + gx) * (R + 1);
          const Real* dbx = gdb + (int64_t(ex) * NG + gx) * (R + 1);
          const Real* by = gb + (int64_t(ey) * NG + gy) * (R + 1);
          const Real* dby = gdb + (int64_t(ey) * NG + gy) * (R + 1);
          const Real* bz = gb + (int64_t(ez) * NG + gz) * (R + 1);
          const Real* dbz = gdb + (int64_t(ez) * NG + gz) * (R + 1);
          Real s = 0, px = 0, py = 0, pz = 0;
#pragma unroll
          for (int cc = 0; cc <= R; ++cc) {
            Real ps = 0, ppx = 0, ppy = 0, ppz = 0;
#pragma unroll
            for (int bb = 0; bb <= R; ++bb) {
              Real rs = 0, rpx = 0, rp = 0;
#pragma unroll
              for (int a = 0; a <= R; ++a) {
                const int li = (cc * TCO + eyl + bb) * TCO + exl + a;
                rs += bx[a] * sS[li];
                rpx += dbx[a] * sP[li];
                rp += bx[a] * sP[li];
              }
              ps += by[bb] * rs;
              ppx += by[bb] * rpx;
              ppy += dby[bb] * rp;
              ppz += by[bb] * rp;
            }
            s += bz[cc] * ps;
            px += bz[cc] * ppx;
            py += bz[cc] * ppy;
            pz += dbz[cc] * ppz;
          }
          const Real xi = gxi[gx], eta = gxi[gy], zeta = gxi[gz];
          const int n0 = eyl * TN + exl;
          auto interp = [&](const Real* arr) {
            const Real lo = (1 - eta) * ((1 - xi) * arr[n0] + xi * arr[n0 + 1]) +
                            eta * ((1 - xi) * arr[n0 + TN] + xi * arr[n0 + TN + 1]);
            const Real* a1 = arr + TN * TN;
            const Real hi = (1 - eta) * ((1 - xi) * a1[n0] + xi * a1[n0 + 1]) +
                            eta * ((1 - xi) * a1[n0 + TN] + xi * a1[n0 + TN + 1]);
            return (1 - zeta) * lo + zeta * hi;
          };
          const Real kk = interp(sK), phi = interp(sF), qin = interp(sQi), qpr = interp(sQp);
          const Real scl = clamp01(s);
          const Real lam_g = powi_or_pow(scl, nexp) * inv_mu_g;
          const Real lam_w = powi_or_pow(Real(1) - scl, nexp) * inv_mu_w;
          const Real fg = lam_g / (lam_g + lam_w);
          const Real qg = qin + fg * qpr;
          const Real w = gw[gx] * gw[gy] * gw[gz];
          const Real tphi = tau / phi;
          f0 = w * (s + tphi * qg);
          const Real c = -w * tphi * lam_g * kk;
          fx = c * px;
          fy = c * py;
          fz = c * (pz + gshift);  // grad p - rho_g g, g = -gravity e_z
        }
        sF0[t] = f0;
        sFx[t] = fx;
        sFy[t] = fy;
        sFz[t] = fz;
      }
      __syncthreads();
      // x test functions: G[a][gyl][gz]
      for (int t = tid; t < TC * GP * NG; t += NT) {
        const int al = t % TC, gyl = (t / TC) % GP, gz = t / (TC * GP);
        const int k = k0 + al;
        Real r0 = 0, ry = 0, rz = 0;
        if (k < nb) {
          for (int ex = k - R; ex <= k; ++ex) {
            if (ex < 0 || ex >= ne) continue;
            const int a = k - ex, exl = ex - c0x;
#pragma unroll
            for (int gx = 0; gx < NG; ++gx) {
              const Real bx = gb[(int64_t(ex) * NG + gx) * (R + 1) + a];
              const Real dbx = gdb[(int64_t(ex) * NG + gx) * (R + 1) + a];
              const int f = (gz * GP + gyl) * GP + exl * NG + gx;
              r0 += bx * sF0[f] + dbx * sFx[f];
              ry += bx * sFy[f];
              rz += bx * sFz[f];
            }
          }
        }
        sG0[t] = r0;
        sGy[t] = ry;
        sGz[t] = rz;
      }
      __syncthreads();
      // y test functions: H[a][b][gz]
      for (int t = tid; t < TC * TC * NG; t += NT) {
        const int al = t % TC, bl = (t / TC) % TC, gz = t / (TC * TC);
        const int l = l0 + bl;
        Real h0 = 0, hz = 0;
        if (l < nb) {
          for (int ey = l - R; ey <= l; ++ey) {
            if (ey < 0 || ey >= ne) continue;
            const int bb = l - ey, eyl = ey - c0y;
#pragma unroll
            for (int gy = 0; gy < NG; ++gy) {
              const Real by = gb[(int64_t(ey) * NG + gy) * (R + 1) + bb];
              const Real dby = gdb[(int64_t(ey) * NG + gy) * (R + 1) + bb];
              const int f = (gz * GP + eyl * NG + gy) * TC + al;
              h0 += by * sG0[f] + dby * sGy[f];
              hz += by * sGz[f];
            }
          }
        }
        sH0[t] = h0;
        sHz[t] = hz;
      }
      __syncthreads();
      // z test functions into the rolling accumulators (c = ez + j)
      if (owner) {
#pragma unroll
        for (int j = 0; j <= R; ++j) {
          Real v = 0;
#pragma unroll
          for (int gz = 0; gz < NG; ++gz) {
            const Real bz = gb[(int64_t(ez) * NG + gz) * (R + 1) + j];
            const Real dbz = gdb[(int64_t(ez) * NG + gz) * (R + 1) + j];
            const int f = (gz * TC + own_b) * TC + own_a;
            v += bz * sH0[f] + dbz * sHz[f];
          }
          acc[j] += v;
        }
      }
    }
    // coefficient c = ez has all its layers once c >= cz0
    if (owner && ez >= cz0 && kx < nb && ly < nb)
      b[int64_t(ez) * nbb + int64_t(ly) * nb + kx] = acc[0];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = acc[j + 1];
    acc[R] = 0;
  }
}

template <typename Real, int R>
void launch_ads3(const Geom& g, const Real* s, const Real* p, const Real* perm,
                 const Real* poro, const Real* qi, const Real* qp, const Real* gb,
                 const Real* gdb, const Real* gxi, const Real* gw, const double* tau, Real iw,
                 Real ig, Real ne, Real gs, Real* b, hipStream_t st) {
  constexpr bool big = sizeof(Real) == 8;
  constexpr int TC = big ? (R == 3 ? 2 : 4) : (R == 3 ? 4 : 8);
  constexpr int ZC = 16;
  dim3 grid(cdiv(g.nb, TC), cdiv(g.nb, TC), cdiv(g.nb, ZC));
  k_ads_assemble3<Real, R, TC, ZC><<<grid, 256, 0, st>>>(g, s, p, perm, poro, qi, qp, gb, gdb,
                                                         gxi, gw, tau, iw, ig, ne, gs, b);
}

template <typename Real>
void launch_ads_assemble(const Geom& g, const Real* s, const Real* p, const Real* perm,
                         const Real* poro, const Real* qi, const Real* qp, const Real* gb,
                         const Real* gdb, const Real* gxi, const Real* gw, const double* tau,
                         double mu_w, double mu_g, double nexp, double gshift, Real* b,
                         hipStream_t st, Batch bz) {
  const double* t = tau;
  const Real iw = Real(1.0 / mu_w), ig = Real(1.0 / mu_g), ne = Real(nexp), gs = Real(gshift);
  if (g.dim == 3) {
    if (g.r == 1)
      launch_ads3<Real, 1>(g, s, p, perm, poro, qi, qp, gb, gdb, gxi, gw, t, iw, ig, ne, gs, b, st);
    else if (g.r == 2)
      launch_ads3<Real, 2>(g, s, p, perm, poro, qi, qp, gb, gdb, gxi, gw, t, iw, ig, ne, gs, b, st);
    else
      launch_ads3<Real, 3>(g, s, p, perm, poro, qi, qp, gb, gdb, gxi, gw, t, iw, ig, ne, gs, b, st);
    return;
  }
  constexpr bool big = sizeof(Real) == 8;
  if (g.r == 1) {
    constexpr int TC = 16;
    dim3 grid(cdiv(g.nb, TC), cdiv(g.nb, TC), bz.n);
    k_ads_assemble2<Real, 1, TC><<<grid, TC * TC, 0, st>>>(g, s, p, perm, poro, qi, qp, gb, gdb, gxi, gw, t, iw, ig, ne, gs, b, bz.zb);
  } else if (g.r == 2) {
    constexpr int TC = big ? 8 : 16;
    dim3 grid(cdiv(g.nb, TC), cdiv(g.nb, TC), bz.n);
    k_ads_assemble2<Real, 2, TC><<<grid, TC * TC, 0, st>>>(g, s, p, perm, poro, qi, qp, gb, gdb, gxi, gw, t, iw, ig, ne, gs, b, bz.zb);
  } else {
    constexpr int TC = 8;
    dim3 grid(cdiv(g.nb, TC), cdiv(g.nb, TC), bz.n);
    k_ads_assemble2<Real, 3, TC><<<grid, TC * TC, 0, st>>>(g, s, p, perm, poro, qi, qp, gb, gdb, gxi, gw, t, iw, ig, ne, gs, b, bz.zb);
  }
}

// ---------------------------------------------------------------------------
// K7f: float64 factorisations (device), converted to the working precision.
// ---------------------------------------------------------------------------
template <typename Real>
__global__ void k_factor_band(const double* __restrict__ band, int n, int r,
                              double* __restrict__ d, Real* __restrict__ lt,
                              Real* __restrict__ inv_d, int* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  // M(j, j+t) = band[j*(r+1)+t]; keep L in float64 in the lt slots of d[n..]
  double* L = d + n;  // n*r entries, L(i, i-t) at L[i*r + t-1]
  for (int j = 0; j < n; ++j) {
    double dj = band[int64_t(j) * (r + 1)];
    for (int k = max(0, j - r); k < j; ++k) {
      const double l = L[int64_t(j) * r + (j - k - 1)];
      dj -= l * l * d[k];
    }
    if (!(dj > 0.0)) {
      *status = 1;
      return;
    }
    d[j] = dj;
    for (int i = j + 1; i <= min(n - 1, j + r); ++i) {
      double mij = band[int64_t(j) * (r + 1) + (i - j)];
      for (int k = max(0, i - r); k < j; ++k)
        mij -= L[int64_t(i) * r + (i - k - 1)] * L[int64_t(j) * r + (j - k - 1)] * d[k];
      L[int64_t(i) * r + (i - j - 1)] = mij / dj;
    }
  }
  for (int j = 0; j < n; ++j) {
    inv_d[j] = Real(1.0 / d[j]);
    for (int t = 0; t < r; ++t) lt[int64_t(j) * r + t] = Real(j - t - 1 >= 0 ? L[int64_t(j) * r + t] : 0.0);
  }
  *status = 0;
}

template <typename Real>
void launch_factor_band(const double* band, int n, int r, double* work_d, Real* lt, Real* inv_d,
                        int* status, hipStream_t st) {
  k_factor_band<Real><<<1, 64, 0, st>>>(band, n, r, work_d, lt, inv_d, status);
}

template <typename Real>
__global__ void k_factor_shifted(const double* __restrict__ shifts, int nlines, int m, int mp,
                                 double scale, Real* __restrict__ lt, Real* __restrict__ inv_d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nlines) return;
  const double diag = scale * (2.0 + shifts[k]), off = -scale;
  double dprev = 0;
  for (int j = 0; j < m; ++j) {
    double dj, l = 0;
    if (j == 0) {
      dj = diag;
    } else {
      l = off / dprev;
      dj = diag - l * l * dprev;
    }
    lt[int64_t(k) * mp + j] = Real(l);
    inv_d[int64_t(k) * mp + j] = Real(1.0 / dj);
    dprev = dj;
  }
}

template <typename Real>
void launch_factor_shifted(const double* shifts, int nlines, int m, int mp, double scale,
                           Real* lt, Real* inv_d, hipStream_t st) {
  k_factor_shifted<Real><<<cdiv(nlines, 64), 64, 0, st>>>(shifts, nlines, m, mp, scale, lt, inv_d);
}

// ---------------------------------------------------------------------------
// one float64 into device memory, stream-ordered (the substep length read by
// a captured step; no host wait)
__global__ void k_set_f64(double* p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

void launch_set_f64(double* p, double v, hipStream_t st) { k_set_f64<<<1, 64, 0, st>>>(p, v); }

// one value per scenario of a batch: p + k zb bytes <- v[k]
struct F64Batch {
  double v[64];
};
__global__ void k_set_f64_batch(double* p, int64_t zb, int n, F64Batch vals) {
  const int k = threadIdx.x;
  if (blockIdx.x == 0 && k < n)
    *reinterpret_cast<double*>(reinterpret_cast<char*>(p) + int64_t(k) * zb) = vals.v[k];
}
void launch_set_f64_batch(double* p, int64_t zb, const double* v, int n, hipStream_t st) {
  for (int k0 = 0; k0 < n; k0 += 64) {
    F64Batch vals{};
    const int cnt = n - k0 < 64 ? n - k0 : 64;
    for (int k = 0; k < cnt; ++k) vals.v[k] = v[k0 + k];
    k_set_f64_batch<<<1, 64, 0, st>>>(
        reinterpret_cast<double*>(reinterpret_cast<char*>(p) + int64_t(k0) * zb), zb, cnt, vals);
  }
}

__global__ void k_bump(long long* t) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *t = *t + 1;
}
void launch_bump(long long* t, hipStream_t st) { k_bump<<<1, 64, 0, st>>>(t); }

template <typename Real>
__global__ void k_fill(Real* p, size_t n, Real v) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
template <typename Real>
void launch_fill(Real* p, size_t n, Real v, hipStream_t st) {
  if (n == 0) return;
  k_fill<Real><<<cdiv(n, 256), 256, 0, st>>>(p, n, v);
}

template <typename Src, typename Dst>
__global__ void k_convert(const Src* in, Dst* out, size_t n) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = Dst(in[i]);
}
template <typename Src, typename Dst>
void launch_convert(const Src* in, Dst* out, size_t n, hipStream_t st) {
  if (n == 0) return;
  k_convert<Src, Dst><<<cdiv(n, 256), 256, 0, st>>>(in, out, n);
}

template <typename Real>
__global__ void k_check_finite(const Real* p, size_t n, int* flag, int64_t zb) {
  p = zofs(p, zb);
  flag = zofs(flag, zb);
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(p[i])) *flag = 1;
}
template <typename Real>
void launch_check_finite(const Real* p, size_t n, int* flag, hipStream_t st, Batch bz) {
  if (n == 0) return;
  k_check_finite<Real><<<dim3(cdiv(n, 256), 1, bz.n), 256, 0, st>>>(p, n, flag, bz.zb);
}

#define CRV_INST(R)                                                                              \
  template void launch_refresh<R>(const Geom&, const R*, const int*, const R*, const R*, double, \
                                  double, double, double, double, R*, R*, R*, hipStream_t,       \
                                  Batch);                                                        \
  template void launch_gravity_rhs<R>(const Geom&, const R*, const R*, const R*, double, R*,     \
                                      hipStream_t, Batch);                                       \
  template void launch_residual<R>(const Geom&, const R*, const R*, const R*, R*, hipStream_t,   \
                                   Batch);                                                       \
  template int launch_adjoint<R>(const Geom&, const R*, const R*, const R*, R*, R*, hipStream_t, \
                                 const R*, const R*, const R*);                                 \
  template void launch_adam_logk<R>(int64_t, R*, R*, R*, const R*, R*, double, double, double,  \
                                    double, const long long*, hipStream_t);                     \
  template void launch_loss_finalize<R>(const R*, int, double*, int, const long long*, int,      \
                                        hipStream_t);                                            \
  template void launch_grad_logperm<R>(const Geom&, const R*, const R*, const R*, const R*, double, \
                                       R*, hipStream_t);                                         \
  template void launch_project<R>(const Geom&, const R*, const R*, R*, hipStream_t, Batch);      \
  template void launch_ads_assemble<R>(const Geom&, const R*, const R*, const R*, const R*,      \
                                       const R*, const R*, const R*, const R*, const R*,         \
                                       const R*, const double*, double, double, double, double,  \
                                       R*, hipStream_t, Batch);                                  \
  template void launch_factor_band<R>(const double*, int, int, double*, R*, R*, int*, hipStream_t); \
  template void launch_factor_shifted<R>(const double*, int, int, int, double, R*, R*, hipStream_t); \
  template void launch_fill<R>(R*, size_t, R, hipStream_t);                                      \
  template void launch_check_finite<R>(const R*, size_t, int*, hipStream_t, Batch);

CRV_INST(float)
CRV_INST(double)
template void launch_convert<double, float>(const double*, float*, size_t, hipStream_t);
template void launch_convert<float, double>(const float*, double*, size_t, hipStream_t);
template void launch_convert<double, double>(const double*, double*, size_t, hipStream_t);
template void launch_fill<int>(int*, size_t, int, hipStream_t);

}  // namespace crv
