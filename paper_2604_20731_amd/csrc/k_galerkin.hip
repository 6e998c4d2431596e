// IGA Galerkin pressure system (the paper's direct-solver path, eq. 15-20),
// 2D: S P = F with S = int alpha grad B . grad B and
// F = int q B + int (g F_b) . grad B (g = -gravity e_y), P = 0 on the boundary
// coefficients, solved by conjugate gradients, preconditioned by the diagonal
// of S or by a scaled Kronecker (fast-diagonalisation) inverse.
//
// S is never assembled.  Its product with a coefficient vector runs on tiles
// of TC x TC coefficients per block: the block stages the coefficients its
// elements touch in LDS, evaluates w alpha grad x at the Gauss points of those
// elements into LDS, and each thread sums its own coefficient's share over its
// support in a fixed order (no atomics); the same pass leaves the block's part
// of x . Sx for the CG step.  Load and diagonal are one-off gathers from
// Gauss-point arrays.  Gauss-point arrays are (Ne (r+1))^2, x fastest;
// coefficient arrays nb^2.
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

// y = S x on a TC x TC tile of coefficients per block (boundary coefficients
// 0); part[2 b] = the tile's share of x . y, part[2 b + 1] = 0
template <typename Real, int R, int TC>
__global__ __launch_bounds__(TC* TC) void k_gal_apply2(Geom g, const Real* __restrict__ x,
                                                      const Real* __restrict__ c,
                                                      const Real* __restrict__ gb,
                                                      const Real* __restrict__ gdb,
                                                      Real* __restrict__ y,
                                                      double* __restrict__ part) {
  constexpr int NG = R + 1;
  constexpr int TE = TC + R;       // elements per tile and axis
  constexpr int TCO = TC + 2 * R;  // coefficients those elements touch
  constexpr int GP = TE * NG;      // Gauss points per axis
  __shared__ Real sX[TCO * TCO], sFx[GP * GP], sFy[GP * GP];
  __shared__ double red[TC * TC];
  const int tid = threadIdx.x;
  const int k0 = blockIdx.x * TC, l0 = blockIdx.y * TC;
  const int c0x = k0 - R, c0y = l0 - R;
  const int nb = g.nb, ne = g.ne, ng = ne * NG;
  for (int t = tid; t < TCO * TCO; t += TC * TC) {
    const int a = c0x + t % TCO, bb = c0y + t / TCO;
    sX[t] = (a >= 0 && a < nb && bb >= 0 && bb < nb) ? x[int64_t(bb) * nb + a] : Real(0);
  }
  __syncthreads();
  for (int t = tid; t < GP * GP; t += TC * TC) {
    const int gxl = t % GP, gyl = t / GP;
    const int exl = gxl / NG, gx = gxl % NG, eyl = gyl / NG, gy = gyl % NG;
    const int ex = c0x + exl, ey = c0y + eyl;
    Real fx = 0, fy = 0;
    if (ex >= 0 && ex < ne && ey >= 0 && ey < ne) {
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
          const Real v = sX[(eyl + b) * TCO + exl + a];
          rx += dbx[a] * v;
          rv += bx[a] * v;
        }
        px += by[b] * rx;
        py += dby[b] * rv;
      }
      const Real cc = c[int64_t(ey * NG + gy) * ng + ex * NG + gx];
      fx = cc * px;
      fy = cc * py;
    }
    sFx[t] = fx;
    sFy[t] = fy;
  }
  __syncthreads();
  const int tx = tid % TC, ty = tid / TC;
  const int k = k0 + tx, l = l0 + ty;
  double xy = 0;
  if (k < nb && l < nb) {
    Real acc = 0;
    if (k > 0 && l > 0 && k < nb - 1 && l < nb - 1) {
      for (int ey = max(l - R, 0); ey <= min(l, ne - 1); ++ey) {
        const int bb = l - ey, eyl = ey - c0y;
        for (int ex = max(k - R, 0); ex <= min(k, ne - 1); ++ex) {
          const int a = k - ex, exl = ex - c0x;
#pragma unroll
          for (int gy = 0; gy < NG; ++gy) {
            const Real by = gb[(int64_t(ey) * NG + gy) * (R + 1) + bb];
            const Real dby = gdb[(int64_t(ey) * NG + gy) * (R + 1) + bb];
#pragma unroll
            for (int gx = 0; gx < NG; ++gx) {
              const Real bx = gb[(int64_t(ex) * NG + gx) * (R + 1) + a];
              const Real dbx = gdb[(int64_t(ex) * NG + gx) * (R + 1) + a];
              const int t = (eyl * NG + gy) * GP + exl * NG + gx;
              acc += dbx * by * sFx[t] + bx * dby * sFy[t];
            }
          }
        }
      }
    }
    y[int64_t(l) * nb + k] = acc;
    xy = double(sX[(ty + R) * TCO + tx + R]) * double(acc);
  }
  const double t = block_sum_n<TC * TC>(xy, red);
  if (tid == 0) {
    const int64_t bid = int64_t(blockIdx.y) * gridDim.x + blockIdx.x;
    part[2 * bid] = t;
    part[2 * bid + 1] = 0;
  }
}

// ---- conjugate-gradient pieces; scalars live on the device (sc[]):
//      0 and 1 rz of consecutive iterations (alternating), 2 pAp, 3 rr, 4 ff
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

// x = 0, r = F and z = r / d, p = z (dg given) or p = 0 (dg null: z comes
// from the Kronecker preconditioner and p = z + b p then sets p = z)
template <typename Real>
__global__ __launch_bounds__(256) void k_pcg_init(int64_t n, const Real* __restrict__ f,
                                                  const Real* __restrict__ dg, Real* __restrict__ x,
                                                  Real* __restrict__ r, Real* __restrict__ z,
                                                  Real* __restrict__ p) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] = 0;
  r[i] = f[i];
  if (dg) {
    z[i] = f[i] / dg[i];
    p[i] = z[i];
  } else {
    p[i] = 0;
  }
}

// a = rz / pAp (rz in slot s_rz): x += a p, r -= a Ap and, with JAC,
// z = r / d and the block's parts of the new r.z and r.r (grid-stride,
// kDotBlocks blocks); without JAC z and the parts are left alone
template <typename Real, bool JAC>
__global__ __launch_bounds__(256) void k_pcg_step1(int64_t n, const double* __restrict__ sc,
                                                   int s_rz, Real* __restrict__ x,
                                                   Real* __restrict__ r, Real* __restrict__ z,
                                                   const Real* __restrict__ p,
                                                   const Real* __restrict__ ap,
                                                   const Real* __restrict__ dg,
                                                   double* __restrict__ part) {
  __shared__ double red[256];
  const Real a = sc[2] != 0.0 ? Real(sc[s_rz] / sc[2]) : Real(0);  // converged exactly: stay
  double s1 = 0, s2 = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    x[i] += a * p[i];
    const Real ri = r[i] - a * ap[i];
    r[i] = ri;
    if constexpr (JAC) {
      const Real zi = ri / dg[i];
      z[i] = zi;
      s1 += double(ri) * double(zi);
      s2 += double(ri) * double(ri);
    }
  }
  if constexpr (!JAC) return;
  const double t1 = block_sum_n<256>(s1, red);
  const double t2 = block_sum_n<256>(s2, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = t1;
    part[2 * blockIdx.x + 1] = t2;
  }
}

// b = rz_new / rz_old: p = z + b p
template <typename Real>
__global__ __launch_bounds__(256) void k_pcg_step2(int64_t n, const double* __restrict__ sc,
                                                   int s_new, int s_old, const Real* __restrict__ z,
                                                   Real* __restrict__ p) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Real b = sc[s_old] != 0.0 ? Real(sc[s_new] / sc[s_old]) : Real(0);
  p[i] = z[i] + b * p[i];
}

// ---- scaled Kronecker (fast-diagonalisation) preconditioner:
//   z = D (V x V) L^-1 (V x V) D r   on the m = nb - 2 interior coefficients
// per axis, with V the orthonormal DST-I basis of size m (padded to mp, a
// multiple of 64), L_ij = k_i m_j + m_i k_j where m_i, k_i are the symbols
// of the uniform B-spline mass and stiffness at the DST-I frequencies (the
// symbol of the constant-coefficient operator K x M + M x K), and
// D = sqrt(d0 / diag S) with d0 the diagonal of that operator, so that
// D S D has the constant-coefficient diagonal.  D, V, L are symmetric and
// positive (semi-)definite, so z = P r is a valid CG preconditioner.  The
// four DST-I products run on the matrix cores; between them the interior
// array is transposed once per axis change.

// w at every Gauss point (the c of the constant-coefficient operator)
template <typename Real, int R>
__global__ __launch_bounds__(256) void k_gal_weights2(Geom g, const Real* __restrict__ gw,
                                                      Real* __restrict__ c) {
  constexpr int NG = R + 1;
  const int ng = g.ne * NG;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(ng) * ng) return;
  c[t] = gw[int(t % ng) % NG] * gw[int(t / ng) % NG];
}

// ksc = sqrt(d0 / diag S) on the interior (d0 held in ksc on entry), 0 on the
// boundary coefficients
template <typename Real>
__global__ __launch_bounds__(256) void k_kron_scalevec(int nb, const Real* __restrict__ dg,
                                                       Real* __restrict__ ksc) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nb) * nb) return;
  const int k = int(t % nb), l = int(t / nb);
  const bool edge = k == 0 || l == 0 || k == nb - 1 || l == nb - 1;
  ksc[t] = edge ? Real(0) : Real(sqrt(ksc[t] / dg[t]));
}

// t[i][j] = (ksc r) at coefficient (i + 1, j + 1) (row i along y), 0 in the
// padding (i or j >= m)
template <typename Real>
__global__ __launch_bounds__(256) void k_kron_in(int nb, int m, int mp, const Real* __restrict__ r,
                                                 const Real* __restrict__ ksc,
                                                 Real* __restrict__ t) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(mp) * mp) return;
  const int i = int(e / mp), j = int(e % mp);
  Real v = 0;
  if (i < m && j < m) {
    const int64_t c = int64_t(i + 1) * nb + j + 1;
    v = ksc[c] * r[c];
  }
  t[e] = v;
}

// z = ksc t on the interior (the inverse of k_kron_in's layout), 0 on the
// boundary coefficients
template <typename Real>
__global__ __launch_bounds__(256) void k_kron_out(int nb, int mp, const Real* __restrict__ t,
                                                  const Real* __restrict__ ksc,
                                                  Real* __restrict__ z) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= int64_t(nb) * nb) return;
  const int k = int(c % nb), l = int(c / nb);
  const bool edge = k == 0 || l == 0 || k == nb - 1 || l == nb - 1;
  z[c] = edge ? Real(0) : ksc[c] * t[int64_t(l - 1) * mp + k - 1];
}

// t[i][j] /= k_i m_j + m_i k_j with sym = (m_0 .. m_mp-1, k_0 .. k_mp-1)
// (padded modes carry m = k = 1 and zero values)
template <typename Real>
__global__ __launch_bounds__(256) void k_kron_scale(int mp, const Real* __restrict__ sym,
                                                    Real* __restrict__ t) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(mp) * mp) return;
  const int i = int(e / mp), j = int(e % mp);
  t[e] /= sym[mp + i] * sym[j] + sym[i] * sym[mp + j];
}

// out = in^T for an mp x mp array (mp a multiple of 32): 32 x 32 tiles
// through LDS, 32 x 8 threads, coalesced on both sides
template <typename Real>
__global__ __launch_bounds__(256) void k_transpose(int mp, const Real* __restrict__ in,
                                                   Real* __restrict__ out) {
  __shared__ Real tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
#pragma unroll
  for (int k = 0; k < 32; k += 8) tile[ty + k][tx] = in[int64_t(r0 + ty + k) * mp + c0 + tx];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 32; k += 8) out[int64_t(c0 + ty + k) * mp + r0 + tx] = tile[tx][ty + k];
}

// z = P r (r and z nb^2 coefficient arrays, boundary 0); the DST-I basis is
// symmetric, so every product is V times an mp x mp array: along y, then
// (transposed) along x, scale, along x, (transposed back) along y
template <typename Real>
static void kron_apply(const GalerkinWork<Real>& w, int nb, const Real* r, Real* z,
                       hipStream_t st) {
  const int m = w.mg, mp = w.mgp;
  const int64_t mp2 = int64_t(mp) * mp;
  const dim3 tgrid(mp / 32, mp / 32);
  k_kron_in<Real><<<cdiv(mp2, 256), 256, 0, st>>>(nb, m, mp, r, w.ksc, w.kt0);
  launch_gemm<Real>(mp, mp, mp, w.kdst, mp, w.kt0, mp, w.kt1, mp, st, w.kdst_pk);
  k_transpose<Real><<<tgrid, 256, 0, st>>>(mp, w.kt1, w.kt0);
  launch_gemm<Real>(mp, mp, mp, w.kdst, mp, w.kt0, mp, w.kt1, mp, st, w.kdst_pk);
  k_kron_scale<Real><<<cdiv(mp2, 256), 256, 0, st>>>(mp, w.ksym, w.kt1);
  launch_gemm<Real>(mp, mp, mp, w.kdst, mp, w.kt1, mp, w.kt0, mp, st, w.kdst_pk);
  k_transpose<Real><<<tgrid, 256, 0, st>>>(mp, w.kt0, w.kt1);
  launch_gemm<Real>(mp, mp, mp, w.kdst, mp, w.kt1, mp, w.kt0, mp, st, w.kdst_pk);
  k_kron_out<Real><<<cdiv(int64_t(nb) * nb, 256), 256, 0, st>>>(nb, mp, w.kt0, w.ksc, z);
}

// tile edge of the operator kernel: 16 (float, r <= 2), else 8 (LDS)
template <typename Real, int R>
constexpr int gal_tc() { return (sizeof(Real) == 4 && R <= 2) ? 16 : 8; }

int64_t galerkin_partials(const Geom& g) {
  const int64_t t = cdiv(g.nb, 8);
  return std::max<int64_t>(kDotBlocks, t * t);
}

template <typename Real, int R>
static void gal_setup(const Geom& g, const GalerkinArgs<Real>& a, hipStream_t st) {
  const int64_t npts = ipow(int64_t(g.ne) * (R + 1), 2);
  k_gal_fields2<Real, R><<<cdiv(npts, 256), 256, 0, st>>>(
      g, a.s, a.perm, a.qi, a.qp, a.gb, a.gxi, a.gw, Real(1.0 / a.mu_w), Real(1.0 / a.mu_g),
      Real(a.nexp), Real(a.rho_w / a.mu_w), Real(a.rho_g / a.mu_g), Real(a.gravity), a.ws.c,
      a.ws.f0, a.gravity != 0.0 ? a.ws.fy : nullptr);
  const int64_t n = int64_t(g.nb) * g.nb;
  k_gal_gather2<Real, R, false><<<cdiv(n, 256), 256, 0, st>>>(
      g, a.ws.f0, nullptr, a.gravity != 0.0 ? a.ws.fy : nullptr, a.gb, a.gdb, a.ws.f);
  k_gal_gather2<Real, R, true><<<cdiv(n, 256), 256, 0, st>>>(g, a.ws.c, nullptr, nullptr, a.gb,
                                                             a.gdb, a.ws.dg);
  const bool kron = a.precond == 1;
  if (kron) {
    // d0 from the diagonal gather with alpha = 1 (f0 is free again)
    k_gal_weights2<Real, R><<<cdiv(npts, 256), 256, 0, st>>>(g, a.gw, a.ws.f0);
    k_gal_gather2<Real, R, true><<<cdiv(n, 256), 256, 0, st>>>(g, a.ws.f0, nullptr, nullptr, a.gb,
                                                               a.gdb, a.ws.ksc);
    k_kron_scalevec<Real><<<cdiv(n, 256), 256, 0, st>>>(g.nb, a.ws.dg, a.ws.ksc);
  }
  k_pcg_init<Real><<<cdiv(n, 256), 256, 0, st>>>(n, a.ws.f, kron ? nullptr : a.ws.dg, a.x, a.ws.r,
                                                 a.ws.z, a.ws.p);
  if (kron) kron_apply<Real>(a.ws, g.nb, a.ws.r, a.ws.z, st);
  k_dot2_part<Real><<<kDotBlocks, 256, 0, st>>>(n, a.ws.r, a.ws.z, a.ws.f, a.ws.f, a.ws.part);
  k_dot2_fin<<<1, 256, 0, st>>>(a.ws.part, kDotBlocks, a.ws.sc, 0, 4);
  // p = z + b 0 = z
  if (kron) k_pcg_step2<Real><<<cdiv(n, 256), 256, 0, st>>>(n, a.ws.sc, 0, 0, a.ws.z, a.ws.p);
}

// iters CG iterations; iteration it starts with rz in slot it & 1
template <typename Real, int R>
static void gal_iters(const Geom& g, const GalerkinArgs<Real>& a, int iters, hipStream_t st) {
  constexpr int TC = gal_tc<Real, R>();
  const int64_t n = int64_t(g.nb) * g.nb;
  const dim3 tiles(cdiv(g.nb, TC), cdiv(g.nb, TC));
  const int ntiles = int(tiles.x * tiles.y);
  for (int it = 0; it < iters; ++it) {
    const int s_old = it & 1, s_new = s_old ^ 1;
    k_gal_apply2<Real, R, TC><<<tiles, TC * TC, 0, st>>>(g, a.ws.p, a.ws.c, a.gb, a.gdb, a.ws.ap,
                                                         a.ws.part);
    k_dot2_fin<<<1, 256, 0, st>>>(a.ws.part, ntiles, a.ws.sc, 2, -1);
    if (a.precond == 1) {
      k_pcg_step1<Real, false><<<kDotBlocks, 256, 0, st>>>(n, a.ws.sc, s_old, a.x, a.ws.r, a.ws.z,
                                                           a.ws.p, a.ws.ap, a.ws.dg, a.ws.part);
      kron_apply<Real>(a.ws, g.nb, a.ws.r, a.ws.z, st);
      k_dot2_part<Real><<<kDotBlocks, 256, 0, st>>>(n, a.ws.r, a.ws.z, a.ws.r, a.ws.r, a.ws.part);
    } else {
      k_pcg_step1<Real, true><<<kDotBlocks, 256, 0, st>>>(n, a.ws.sc, s_old, a.x, a.ws.r, a.ws.z,
                                                          a.ws.p, a.ws.ap, a.ws.dg, a.ws.part);
    }
    k_dot2_fin<<<1, 256, 0, st>>>(a.ws.part, kDotBlocks, a.ws.sc, s_new, 3);
    k_pcg_step2<Real><<<cdiv(n, 256), 256, 0, st>>>(n, a.ws.sc, s_new, s_old, a.ws.z, a.ws.p);
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
