// IGA Galerkin pressure system (the paper's direct-solver path, eq. 15-20),
// 2D: S P = F with S = int alpha grad B . grad B and
// F = int q B + int (g F_b) . grad B (g = -gravity e_y), P = 0 on the boundary
// coefficients, solved by conjugate gradients with the diagonal of S as the
// preconditioner.
//
// S is never assembled.  Its product with a coefficient vector is two passes:
// the gradient of the spline at every Gauss point times w alpha there (one
// thread per Gauss point), then, for every coefficient, the sum over the
// Gauss points of its support of that flux against the basis gradient (one
// thread per coefficient, fixed order, no atomics).  Load and diagonal use the
// same gather.  Gauss-point arrays are (Ne (r+1))^2, x fastest; coefficient
// arrays nb^2.
#include "kernels.h"

namespace crv {

// w alpha, w q and -gravity w F_b at every Gauss point (S from the spline, K
// and q Q1-interpolated from the nodes, as in the saturation update)
template <typename Real, int R>
__global__ __launch_bounds__(256) void k_gal_fields2(
    Geom g, const Real* __restrict__ sc, const Real* __restrict__ perm, const Real* __restrict__ qi,
    const Real* __restrict__ qp, const Real* __restrict__ gb, const Real* __restrict__ gxi,
    const Real* __restrict__ gw, Real inv_mu_w, Real inv_mu_g, Real nexp, Real rw_mu, Real rg_mu,
    Real gravity, Real* __restrict__ c, Real* __restrict__ f0, Real* __restrict__ fy) {
  constexpr int NG = R + 1;
  const int ng = g.ne * NG;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(ng) * ng) return;
  const int gxl = int(t % ng), gyl = int(t / ng);
  const int ex = gxl / NG, gx = gxl % NG, ey = gyl / NG, gy = gyl % NG;
  const Real* bx = gb + (int64_t(ex) * NG + gx) * (R + 1);
  const Real* by = gb + (int64_t(ey) * NG + gy) * (R + 1);
  Real s = 0;
#pragma unroll
  for (int b = 0; b <= R; ++b) {
    Real row = 0;
#pragma unroll
    for (int a = 0; a <= R; ++a) row += bx[a] * sc[int64_t(ey + b) * g.nb + ex + a];
    s += by[b] * row;
  }
  const Real xi = gxi[gx], eta = gxi[gy];
  const int64_t n00 = int64_t(ey) * g.n + ex;
  auto q1 = [&](const Real* a) {
    return (1 - xi) * (1 - eta) * a[n00] + xi * (1 - eta) * a[n00 + 1] +
           (1 - xi) * eta * a[n00 + g.n] + xi * eta * a[n00 + g.n + 1];
  };
  const Real kk = q1(perm);
  const Real scl = clamp01(s);
  const Real krw = powi_or_pow(Real(1) - scl, nexp), krg = powi_or_pow(scl, nexp);
  const Real w = gw[gx] * gw[gy];
  c[t] = w * kk * (krw * inv_mu_w + krg * inv_mu_g);
  f0[t] = w * (q1(qi) + q1(qp));
  if (fy) fy[t] = -gravity * w * kk * (krw * rw_mu + krg * rg_mu);
}

// vx = c d_x x, vy = c d_y x at every Gauss point
template <typename Real, int R>
__global__ __launch_bounds__(256) void k_gal_grad2(Geom g, const Real* __restrict__ x,
                                                   const Real* __restrict__ c,
                                                   const Real* __restrict__ gb,
                                                   const Real* __restrict__ gdb,
                                                   Real* __restrict__ vx, Real* __restrict__ vy) {
  constexpr int NG = R + 1;
  const int ng = g.ne * NG;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(ng) * ng) return;
  const int gxl = int(t % ng), gyl = int(t / ng);
  const int ex = gxl / NG, gx = gxl % NG, ey = gyl / NG, gy = gyl % NG;
  const Real* bx = gb + (int64_t(ex) * NG + gx) * (R + 1);
  const Real* dbx = gdb + (int64_t(ex) * NG + gx) * (R + 1);
  const Real* by = gb + (int64_t(ey) * NG + gy) * (R + 1);
  const Real* dby = gdb + (int64_t(ey) * NG + gy) * (R + 1);
  Real px = 0, py = 0;
#pragma unroll
  for (int b = 0; b <= R; ++b) {
    Real rx = 0, rv = 0;
#pragma unroll
    for (int a = 0; a <= R; ++a) {
      const Real v = x[int64_t(ey + b) * g.nb + ex + a];
      rx += dbx[a] * v;
      rv += bx[a] * v;
    }
    px += by[b] * rx;
    py += dby[b] * rv;
  }
  const Real cc = c[t];
  vx[t] = cc * px;
  vy[t] = cc * py;
}

// out_kl = sum over the Gauss points of B_kl's support of
//   DIAG = false: v0 B + vx d_x B + vy d_y B   (v0, vx, vy nullable)
//   DIAG = true:  c (d_x B^2 + d_y B^2)        (c passed as v0)
// Boundary coefficients get 0 (1 for the diagonal), which keeps every CG
// vector zero there.
template <typename Real, int R, bool DIAG>
__global__ __launch_bounds__(256) void k_gal_gather2(Geom g, const Real* __restrict__ v0,
                                                     const Real* __restrict__ vx,
                                                     const Real* __restrict__ vy,
                                                     const Real* __restrict__ gb,
                                                     const Real* __restrict__ gdb,
                                                     Real* __restrict__ out) {
  constexpr int NG = R + 1;
  const int nb = g.nb, ne = g.ne, ng = ne * NG;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nb) * nb) return;
  const int k = int(t % nb), l = int(t / nb);
  if (k == 0 || l == 0 || k == nb - 1 || l == nb - 1) {
    out[t] = DIAG ? Real(1) : Real(0);
    return;
  }
  Real acc = 0;
  for (int ey = max(l - R, 0); ey <= min(l, ne - 1); ++ey) {
    const int bb = l - ey;
    for (int ex = max(k - R, 0); ex <= min(k, ne - 1); ++ex) {
      const int a = k - ex;
#pragma unroll
      for (int gy = 0; gy < NG; ++gy) {
        const Real by = gb[(int64_t(ey) * NG + gy) * (R + 1) + bb];
        const Real dby = gdb[(int64_t(ey) * NG + gy) * (R + 1) + bb];
#pragma unroll
        for (int gx = 0; gx < NG; ++gx) {
          const Real bx = gb[(int64_t(ex) * NG + gx) * (R + 1) + a];
          const Real dbx = gdb[(int64_t(ex) * NG + gx) * (R + 1) + a];
          const int64_t i = int64_t(ey * NG + gy) * ng + ex * NG + gx;
          if constexpr (DIAG) {
            acc += v0[i] * (dbx * dbx * by * by + bx * bx * dby * dby);
          } else {
            if (v0) acc += v0[i] * bx * by;
            if (vx) acc += vx[i] * dbx * by;
            if (vy) acc += vy[i] * bx * dby;
          }
        }
      }
    }
  }
  out[t] = acc;
}

// ---- conjugate-gradient pieces; scalars live on the device (sc[]):
//      0 rz, 1 rz_new, 2 pAp, 3 rr, 4 ff
constexpr int kDotBlocks = 256;

// fixed-order partial sums of a.b and (if c) c.d, double accumulation
template <typename Real>
__global__ __launch_bounds__(256) void k_dot2_part(int64_t n, const Real* __restrict__ a,
                                                   const Real* __restrict__ b,
                                                   const Real* __restrict__ c,
                                                   const Real* __restrict__ d,
                                                   double* __restrict__ part) {
  __shared__ double red[256];
  double s1 = 0, s2 = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    s1 += double(a[i]) * double(b[i]);
    if (c) s2 += double(c[i]) * double(d[i]);
  }
  const double t1 = block_sum_n<256>(s1, red);
  const double t2 = block_sum_n<256>(s2, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = t1;
    part[2 * blockIdx.x + 1] = t2;
  }
}

__global__ __launch_bounds__(256) void k_dot2_fin(const double* __restrict__ part, int nparts,
                                                  double* __restrict__ sc, int slot1, int slot2) {
  __shared__ double red[256];
  double s1 = 0, s2 = 0;
  for (int i = threadIdx.x; i < nparts; i += 256) {
    s1 += part[2 * i];
    s2 += part[2 * i + 1];
  }
  const double t1 = block_sum_n<256>(s1, red);
  const double t2 = block_sum_n<256>(s2, red);
  if (threadIdx.x == 0) {
    sc[slot1] = t1;
    if (slot2 >= 0) sc[slot2] = t2;
  }
}

// x = 0, r = F, z = r / d, p = z
template <typename Real>
__global__ __launch_bounds__(256) void k_pcg_init(int64_t n, const Real* __restrict__ f,
                                                  const Real* __restrict__ dg, Real* __restrict__ x,
                                                  Real* __restrict__ r, Real* __restrict__ z,
                                                  Real* __restrict__ p) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] = 0;
  r[i] = f[i];
  z[i] = f[i] / dg[i];
  p[i] = z[i];
}

// a = rz / pAp: x += a p, r -= a Ap, z = r / d
template <typename Real>
__global__ __launch_bounds__(256) void k_pcg_step1(int64_t n, const double* __restrict__ sc,
                                                   Real* __restrict__ x, Real* __restrict__ r,
                                                   Real* __restrict__ z, const Real* __restrict__ p,
                                                   const Real* __restrict__ ap,
                                                   const Real* __restrict__ dg) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Real a = sc[2] != 0.0 ? Real(sc[0] / sc[2]) : Real(0);  // converged exactly: stay
  x[i] += a * p[i];
  const Real ri = r[i] - a * ap[i];
  r[i] = ri;
  z[i] = ri / dg[i];
}

// b = rz_new / rz: p = z + b p
template <typename Real>
__global__ __launch_bounds__(256) void k_pcg_step2(int64_t n, const double* __restrict__ sc,
                                                   const Real* __restrict__ z, Real* __restrict__ p) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Real b = sc[0] != 0.0 ? Real(sc[1] / sc[0]) : Real(0);
  p[i] = z[i] + b * p[i];
}

__global__ void k_pcg_shift(double* sc) { sc[0] = sc[1]; }

template <typename Real, int R>
static void gal_fields(const Geom& g, const GalerkinArgs<Real>& a, hipStream_t st) {
  const int64_t npts = ipow(int64_t(g.ne) * (R + 1), 2);
  k_gal_fields2<Real, R><<<cdiv(npts, 256), 256, 0, st>>>(
      g, a.s, a.perm, a.qi, a.qp, a.gb, a.gxi, a.gw, Real(1.0 / a.mu_w), Real(1.0 / a.mu_g),
      Real(a.nexp), Real(a.rho_w / a.mu_w), Real(a.rho_g / a.mu_g), Real(a.gravity), a.ws.c,
      a.ws.f0, a.gravity != 0.0 ? a.ws.fy : nullptr);
  const int64_t nc = int64_t(g.nb) * g.nb;
  k_gal_gather2<Real, R, false><<<cdiv(nc, 256), 256, 0, st>>>(
      g, a.ws.f0, nullptr, a.gravity != 0.0 ? a.ws.fy : nullptr, a.gb, a.gdb, a.ws.f);
  k_gal_gather2<Real, R, true><<<cdiv(nc, 256), 256, 0, st>>>(g, a.ws.c, nullptr, nullptr, a.gb,
                                                              a.gdb, a.ws.dg);
}

template <typename Real, int R>
static void gal_apply(const Geom& g, const GalerkinArgs<Real>& a, const Real* x, Real* y,
                      hipStream_t st) {
  const int64_t npts = ipow(int64_t(g.ne) * (R + 1), 2);
  k_gal_grad2<Real, R><<<cdiv(npts, 256), 256, 0, st>>>(g, x, a.ws.c, a.gb, a.gdb, a.ws.vx, a.ws.vy);
  const int64_t nc = int64_t(g.nb) * g.nb;
  k_gal_gather2<Real, R, false><<<cdiv(nc, 256), 256, 0, st>>>(g, nullptr, a.ws.vx, a.ws.vy, a.gb,
                                                               a.gdb, y);
}

template <typename Real>
static void dot2(int64_t n, const Real* x1, const Real* y1, const Real* x2, const Real* y2,
                 double* part, double* sc, int s1, int s2, hipStream_t st) {
  k_dot2_part<Real><<<kDotBlocks, 256, 0, st>>>(n, x1, y1, x2, y2, part);
  k_dot2_fin<<<1, 256, 0, st>>>(part, kDotBlocks, sc, s1, s2);
}

template <typename Real, int R>
static void gal_setup(const Geom& g, const GalerkinArgs<Real>& a, hipStream_t st) {
  gal_fields<Real, R>(g, a, st);
  const int64_t n = int64_t(g.nb) * g.nb;
  k_pcg_init<Real><<<cdiv(n, 256), 256, 0, st>>>(n, a.ws.f, a.ws.dg, a.x, a.ws.r, a.ws.z, a.ws.p);
  dot2<Real>(n, a.ws.r, a.ws.z, a.ws.f, a.ws.f, a.ws.part, a.ws.sc, 0, 4, st);
}

template <typename Real, int R>
static void gal_iters(const Geom& g, const GalerkinArgs<Real>& a, int iters, hipStream_t st) {
  const int64_t n = int64_t(g.nb) * g.nb;
  for (int it = 0; it < iters; ++it) {
    gal_apply<Real, R>(g, a, a.ws.p, a.ws.ap, st);
    dot2<Real>(n, a.ws.p, a.ws.ap, static_cast<const Real*>(nullptr), static_cast<const Real*>(nullptr),
               a.ws.part, a.ws.sc, 2, -1, st);
    k_pcg_step1<Real><<<cdiv(n, 256), 256, 0, st>>>(n, a.ws.sc, a.x, a.ws.r, a.ws.z, a.ws.p, a.ws.ap,
                                                    a.ws.dg);
    dot2<Real>(n, a.ws.r, a.ws.z, a.ws.r, a.ws.r, a.ws.part, a.ws.sc, 1, 3, st);
    k_pcg_step2<Real><<<cdiv(n, 256), 256, 0, st>>>(n, a.ws.sc, a.ws.z, a.ws.p);
    k_pcg_shift<<<1, 1, 0, st>>>(a.ws.sc);
  }
}

template <typename Real>
void launch_galerkin_setup(const Geom& g, const GalerkinArgs<Real>& a, hipStream_t st) {
  if (g.r == 1) gal_setup<Real, 1>(g, a, st);
  else if (g.r == 2) gal_setup<Real, 2>(g, a, st);
  else gal_setup<Real, 3>(g, a, st);
}

template <typename Real>
void launch_galerkin_iters(const Geom& g, const GalerkinArgs<Real>& a, int iters, hipStream_t st) {
  if (g.r == 1) gal_iters<Real, 1>(g, a, iters, st);
  else if (g.r == 2) gal_iters<Real, 2>(g, a, iters, st);
  else gal_iters<Real, 3>(g, a, iters, st);
}

template void launch_galerkin_setup<float>(const Geom&, const GalerkinArgs<float>&, hipStream_t);
template void launch_galerkin_setup<double>(const Geom&, const GalerkinArgs<double>&, hipStream_t);
template void launch_galerkin_iters<float>(const Geom&, const GalerkinArgs<float>&, int, hipStream_t);
template void launch_galerkin_iters<double>(const Geom&, const GalerkinArgs<double>&, int, hipStream_t);

}  // namespace crv
