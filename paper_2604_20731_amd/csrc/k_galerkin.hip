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

// CG scalars on the device (layout below): converged when r.r (slot 3) is at
// or under the threshold (slot 6); slot 5 the running iteration's stop flag
__device__ inline bool cg_converged(const double* sc) { return sc[3] <= sc[6]; }

// blocks of the update kernels (each leaves one (r.z, r.r) pair)
constexpr int kDotBlocks = 256;

// sum over i < np of part[2 i + j] by a block of NTH threads (flat index),
// in a fixed order (every block alike)
template <int NTH>
__device__ inline double sum_pairs_n(const double* __restrict__ part, int np, int j,
                                     double* red) {
  double s = 0;
  for (int i = threadIdx.x; i < np; i += NTH) s += part[2 * i + j];
  return block_sum_n<NTH>(s, red);
}

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

// The conjugate-gradient iteration's first step: from the previous update's
// (r.z, r.r) pairs in part2 (summed by every block alike) the convergence
// test (r.r <= sc[6]: the block returns; block 0 records r.r in sc[3], r.z in
// sc[s_new] and the stop flag in sc[5]), then the direction
// x = z + b p_old with b = r.z / sc[s_old] (0 when that is 0), written to
// p_new for the tile's own coefficients, and y = S x on a TC x TC tile of
// interior coefficients per block (the tiles cover coefficients 1 .. nb-2
// per axis; y and p_new on the boundary coefficients are 0 and never
// written here: the set-up zeroes them); part[2 b] = the tile's share of
// x . y, part[2 b + 1] = 0.  The block
// stages the coefficients its TE x TE elements touch and the 1D basis tables
// of those elements in LDS, then works by sum factorisation (one axis at a
// time, no atomics, fixed summation order):
//   Tx = (d_x B) X, Tv = B X along x            [coefficient rows x Gauss x]
//   Fx = c (B Tx), Fy = c ((d_y B) Tv) along y  [Gauss y x Gauss x]
//   Ux = B Fx, Uy = (d_y B) Fy along y          [tile rows x Gauss x]
//   y = (d_x B) Ux + B Uy along x               [tile rows x tile columns]
// with c = w alpha at the Gauss points.  Tables and fluxes of elements
// outside the mesh are 0, so every sum runs over its full local range.
template <typename Real, int R, int TC>
__global__ __launch_bounds__(TC* TC) void k_gal_apply2(
    Geom g, const Real* __restrict__ z, const Real* __restrict__ p_old, Real* __restrict__ p_new,
    const Real* __restrict__ c, const Real* __restrict__ gb, const Real* __restrict__ gdb,
    Real* __restrict__ y, double* __restrict__ part, const double* __restrict__ part2,
    double* __restrict__ sc, int s_new, int s_old, int ntx, int ntiles) {
  // Workgroups are dealt round-robin over the 8 XCDs: block b takes tile
  // (b % 8) * per + b / 8, so each XCD (one L2) works through a contiguous
  // band of tile rows and neighbouring tiles share their halo in its L2;
  // the grid is 8 per blocks, those past the last tile leave at once
  const int per = int(gridDim.x) / 8;
  const int tile = int(blockIdx.x % 8) * per + int(blockIdx.x / 8);
  if (tile >= ntiles) return;
  constexpr int NG = R + 1;
  constexpr int NT = NG * (R + 1);  // table entries per element
  constexpr int TE = TC + R;        // elements per tile and axis
  constexpr int TCO = TC + 2 * R;   // coefficients those elements touch
  constexpr int GP = TE * NG;       // Gauss points per axis
  constexpr int NTH = TC * TC;
  constexpr int NW1 = 2 * TCO * GP, NW2 = 2 * TC * GP;  // Tx/Tv, then Ux/Uy
  __shared__ Real sX[TCO * TCO], sFx[GP * GP], sFy[GP * GP];
  __shared__ Real sW[NW1 > NW2 ? NW1 : NW2];
  __shared__ Real sB[4][TE * NT];  // B and d B along x, then along y
  __shared__ double red[NTH];
  const int tid = threadIdx.x;
  const double rz = sum_pairs_n<NTH>(part2, kDotBlocks, 0, red);
  const double rr = sum_pairs_n<NTH>(part2, kDotBlocks, 1, red);
  const bool stop = rr <= sc[6];
  const double old = sc[s_old];
  if (tile == 0 && tid == 0) {
    sc[3] = rr;
    sc[s_new] = rz;
    sc[5] = stop ? 1.0 : 0.0;
  }
  if (stop) return;
  const Real bdir = old != 0.0 ? Real(rz / old) : Real(0);
  const int k0 = 1 + (tile % ntx) * TC, l0 = 1 + (tile / ntx) * TC;
  const int c0x = k0 - R, c0y = l0 - R;
  const int nb = g.nb, ne = g.ne, ng = ne * NG;
  for (int t = tid; t < TCO * TCO; t += NTH) {
    const int a = c0x + t % TCO, bb = c0y + t / TCO;
    Real v = 0;
    if (a >= 0 && a < nb && bb >= 0 && bb < nb) {
      const int64_t ci = int64_t(bb) * nb + a;
      v = z[ci] + bdir * p_old[ci];
    }
    sX[t] = v;
  }
  for (int t = tid; t < TE * NT; t += NTH) {
    const int el = t / NT, r = t % NT;
    const int ex = c0x + el, ey = c0y + el;
    const bool okx = ex >= 0 && ex < ne, oky = ey >= 0 && ey < ne;
    sB[0][t] = okx ? gb[int64_t(ex) * NT + r] : Real(0);
    sB[1][t] = okx ? gdb[int64_t(ex) * NT + r] : Real(0);
    sB[2][t] = oky ? gb[int64_t(ey) * NT + r] : Real(0);
    sB[3][t] = oky ? gdb[int64_t(ey) * NT + r] : Real(0);
  }
  __syncthreads();
  Real* sTx = sW;
  Real* sTv = sW + TCO * GP;
  for (int t = tid; t < TCO * GP; t += NTH) {
    const int row = t / GP, gxl = t % GP, exl = gxl / NG, gx = gxl % NG;
    const Real* xr = sX + row * TCO + exl;
    const Real* bx = sB[0] + exl * NT + gx * (R + 1);
    const Real* dbx = sB[1] + exl * NT + gx * (R + 1);
    Real tx = 0, tv = 0;
#pragma unroll
    for (int a = 0; a <= R; ++a) {
      tx += dbx[a] * xr[a];
      tv += bx[a] * xr[a];
    }
    sTx[t] = tx;
    sTv[t] = tv;
  }
  __syncthreads();
  for (int t = tid; t < GP * GP; t += NTH) {
    const int gxl = t % GP, gyl = t / GP;
    const int exl = gxl / NG, eyl = gyl / NG, gy = gyl % NG;
    const int ex = c0x + exl, ey = c0y + eyl;
    Real fx = 0, fy = 0;
    if (ex >= 0 && ex < ne && ey >= 0 && ey < ne) {
      const Real* by = sB[2] + eyl * NT + gy * (R + 1);
      const Real* dby = sB[3] + eyl * NT + gy * (R + 1);
      Real px = 0, py = 0;
#pragma unroll
      for (int b = 0; b <= R; ++b) {
        px += by[b] * sTx[(eyl + b) * GP + gxl];
        py += dby[b] * sTv[(eyl + b) * GP + gxl];
      }
      const Real cc = c[int64_t(ey * NG + gy) * ng + ex * NG + gxl % NG];
      fx = cc * px;
      fy = cc * py;
    }
    sFx[t] = fx;
    sFy[t] = fy;
  }
  __syncthreads();
  // tile row ly (coefficient l0 + ly) meets local elements ly .. ly + R, as
  // basis function R - j of element ly + j
  Real* sUx = sW;
  Real* sUy = sW + TC * GP;
  for (int t = tid; t < TC * GP; t += NTH) {
    const int ly = t / GP, gxl = t % GP;
    Real ux = 0, uy = 0;
#pragma unroll
    for (int j = 0; j <= R; ++j) {
      const int eyl = ly + j;
#pragma unroll
      for (int gy = 0; gy < NG; ++gy) {
        const int tb = eyl * NT + gy * (R + 1) + R - j;
        const int f = (eyl * NG + gy) * GP + gxl;
        ux += sB[2][tb] * sFx[f];
        uy += sB[3][tb] * sFy[f];
      }
    }
    sUx[t] = ux;
    sUy[t] = uy;
  }
  __syncthreads();
  const int tx = tid % TC, ty = tid / TC;
  const int k = k0 + tx, l = l0 + ty;
  double xy = 0;
  if (k < nb - 1 && l < nb - 1) {
    p_new[int64_t(l) * nb + k] = sX[(ty + R) * TCO + tx + R];
    Real acc = 0;
#pragma unroll
    for (int j = 0; j <= R; ++j) {
      const int exl = tx + j;
#pragma unroll
      for (int gx = 0; gx < NG; ++gx) {
        const int tb = exl * NT + gx * (R + 1) + R - j;
        const int u = ty * GP + exl * NG + gx;
        acc += sB[1][tb] * sUx[u] + sB[0][tb] * sUy[u];
      }
    }
    y[int64_t(l) * nb + k] = acc;
    xy = double(sX[(ty + R) * TCO + tx + R]) * double(acc);
  }
  const double t = block_sum_n<TC * TC>(xy, red);
  if (tid == 0) {
    part[2 * tile] = t;
    part[2 * tile + 1] = 0;
  }
}

// ---- conjugate-gradient pieces.  Scalars on the device (sc[]): 0 and 1 the
// r.z of consecutive iterations (alternating slots), 3 r.r, 4 F.F, 5 the
// stop flag of the running iteration, 6 the threshold rtol^2 F.F, 7 the
// iterations done.  An iteration is: operator (convergence test, direction
// p = z + b p_old into the other of two direction arrays, p.Ap partials),
// update (x, r; with the diagonal also z and the (r.z, r.r) pairs), and with
// the Kronecker preconditioner its four products and the scatter with the
// pairs.  Once r.r is at or under the threshold the operator sets the flag
// and every kernel of that and later iterations returns at once, so
// iterations after convergence cost only their launches and the count in
// slot 7 is exact.  The operator leaves one partial of p.Ap per tile in
// part, the update kernels one (r.z, r.r) pair per block in part2; a kernel
// that needs such a sum adds the partials itself, every block in the same
// fixed order, so all blocks hold the same value and no reduction launch
// sits between the steps.
// sum over i < np of part[2 i + j] (blocks of 256 threads; every block alike)
__device__ inline double sum_pairs(const double* __restrict__ part, int np, int j,
                                   double* red) {
  return sum_pairs_n<256>(part, np, j, red);
}

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

// sc[slot1], sc[slot2] = the two sums of nparts pairs (set-up only)
__global__ __launch_bounds__(256) void k_dot2_fin(const double* __restrict__ part, int nparts,
                                                  double* __restrict__ sc, int slot1, int slot2) {
  __shared__ double red[256];
  const double t1 = sum_pairs(part, nparts, 0, red);
  const double t2 = sum_pairs(part, nparts, 1, red);
  if (threadIdx.x == 0) {
    sc[slot1] = t1;
    sc[slot2] = t2;
  }
}

template <typename Real>
__global__ __launch_bounds__(256) void k_zero(int64_t n, Real* __restrict__ a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

__device__ inline bool on_edge(int k, int l, int nb) {
  return k == 0 || l == 0 || k == nb - 1 || l == nb - 1;
}

// x = 0, r = F, p = 0 and either z = r / d (dg given) or the Kronecker
// preconditioner's input t = ksc F on the interior (dg null)
template <typename Real>
__global__ __launch_bounds__(256) void k_pcg_init(int nb, int mp, const Real* __restrict__ f,
                                                  const Real* __restrict__ dg,
                                                  const Real* __restrict__ ksc,
                                                  Real* __restrict__ x, Real* __restrict__ r,
                                                  Real* __restrict__ z, Real* __restrict__ p,
                                                  Real* __restrict__ t) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(nb) * nb) return;
  x[i] = 0;
  r[i] = f[i];
  p[i] = 0;
  if (dg) {
    z[i] = f[i] / dg[i];
  } else {
    const int k = int(i % nb), l = int(i / nb);
    if (!on_edge(k, l, nb)) t[int64_t(l - 1) * mp + k - 1] = ksc[i] * f[i];
  }
}

// Unless this iteration's operator set the stop flag: count the iteration,
// p.Ap from the operator's ntiles partials, a = rz / pAp (rz in slot s_rz):
// x += a p, r -= a Ap, then
//   JAC:  z = r / d and this block's (r.z, r.r) pair in part2;
//   else: the Kronecker preconditioner's input t = ksc r on the interior
// (grid-stride, kDotBlocks blocks of 256)
template <typename Real, bool JAC>
__global__ __launch_bounds__(256) void k_pcg_step1(
    int nb, int mp, double* __restrict__ sc, int s_rz, const double* __restrict__ part,
    int ntiles, Real* __restrict__ x, Real* __restrict__ r, Real* __restrict__ z,
    const Real* __restrict__ p, const Real* __restrict__ ap, const Real* __restrict__ dg,
    const Real* __restrict__ ksc, Real* __restrict__ t, double* __restrict__ part2) {
  __shared__ double red[256];
  if (sc[5] != 0.0) return;  // set by this iteration's operator
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[7] += 1.0;
  const double pap = sum_pairs(part, ntiles, 0, red);
  const Real a = pap != 0.0 ? Real(sc[s_rz] / pap) : Real(0);  // converged exactly: stay
  const int64_t n = int64_t(nb) * nb;
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
    } else {
      const int k = int(i % nb), l = int(i / nb);
      if (!on_edge(k, l, nb)) t[int64_t(l - 1) * mp + k - 1] = ksc[i] * ri;
    }
  }
  if constexpr (!JAC) return;
  const double t1 = block_sum_n<256>(s1, red);
  const double t2 = block_sum_n<256>(s2, red);
  if (threadIdx.x == 0) {
    part2[2 * blockIdx.x] = t1;
    part2[2 * blockIdx.x + 1] = t2;
  }
}

// ---- scaled Kronecker (fast-diagonalisation) preconditioner:
//   z = D (V x V) L^-1 (V x V) D r   on the m = nb - 2 interior coefficients
// per axis, with V the orthonormal DST-I basis of size m (padded to mp, a
// multiple of 64), L_ij = k_i m_j + m_i k_j where m_i, k_i are the symbols
// of the uniform B-spline mass and stiffness at the DST-I frequencies (the
// symbol of the constant-coefficient operator K x M + M x K), and
// D = sqrt(d0 / diag S) with d0 the diagonal of that operator, so that
// D S D has the constant-coefficient diagonal.  D, V, L are symmetric and
// positive definite on the interior, so z = P r is a valid CG
// preconditioner.  The input t0 = D r (row i along y; padding 0, written once)
// comes from the update kernel; four DST-I products on the matrix cores,
// whose epilogues transpose or divide by L:
//   t1 = (V t0)^T,  t2 = (V t1) / L,  t1 = (V t2)^T,  t2 = V t1,
// and the last kernel scatters z = D t2 with the (r.z, r.r) pairs.  The
// padded rows and columns of every product are exactly 0 (V's are).

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
  ksc[t] = on_edge(int(t % nb), int(t / nb), nb) ? Real(0) : Real(sqrt(ksc[t] / dg[t]));
}

// z = ksc t on the interior, 0 on the boundary, and this block's (r.z, r.r)
// pair in part2 (grid-stride, kDotBlocks blocks of 256)
template <typename Real>
__global__ __launch_bounds__(256) void k_kron_out_dot(int nb, int mp, const Real* __restrict__ t,
                                                      const Real* __restrict__ ksc,
                                                      const Real* __restrict__ r,
                                                      Real* __restrict__ z,
                                                      double* __restrict__ part2,
                                                      const double* __restrict__ sc) {
  if (sc && cg_converged(sc)) return;
  __shared__ double red[256];
  const int64_t n = int64_t(nb) * nb;
  double s1 = 0, s2 = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const int k = int(i % nb), l = int(i / nb);
    const Real zi = on_edge(k, l, nb) ? Real(0) : ksc[i] * t[int64_t(l - 1) * mp + k - 1];
    const Real ri = r[i];
    z[i] = zi;
    s1 += double(ri) * double(zi);
    s2 += double(ri) * double(ri);
  }
  const double t1 = block_sum_n<256>(s1, red);
  const double t2 = block_sum_n<256>(s2, red);
  if (threadIdx.x == 0) {
    part2[2 * blockIdx.x] = t1;
    part2[2 * blockIdx.x + 1] = t2;
  }
}

// t0 -> t2 = (V x V) L^-1 (V x V) t0 (the four products); skipped once the
// CG scalars sc (nullable: never skipped) show convergence
template <typename Real>
static void kron_products(const GalerkinWork<Real>& w, const double* sc, hipStream_t st) {
  const int mp = w.mgp;
  const double* skip = sc ? sc + 3 : nullptr;  // skip[0] = r.r, skip[3] = the threshold
  launch_gemm_sq_epi<Real>(mp, w.kdst, w.kt0, w.kt1, 1, w.ksym, st, w.kdst_pk, skip);
  launch_gemm_sq_epi<Real>(mp, w.kdst, w.kt1, w.kt2, 2, w.ksym, st, w.kdst_pk, skip);
  launch_gemm_sq_epi<Real>(mp, w.kdst, w.kt2, w.kt1, 1, w.ksym, st, w.kdst_pk, skip);
  launch_gemm_sq_epi<Real>(mp, w.kdst, w.kt1, w.kt2, 0, w.ksym, st, w.kdst_pk, skip);
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
  const GalerkinWork<Real>& w = a.ws;
  // the operator writes only interior entries: the boundary ones of Ap and of
  // both direction arrays stay 0 (p_old of the first iteration is all 0)
  k_zero<Real><<<cdiv(n, 256), 256, 0, st>>>(n, w.ap);
  k_zero<Real><<<cdiv(n, 256), 256, 0, st>>>(n, w.p2);
  if (a.precond == 1) {
    const int64_t mp2 = int64_t(w.mgp) * w.mgp;
    // d0 from the diagonal gather with alpha = 1 (f0 is free again)
    k_gal_weights2<Real, R><<<cdiv(npts, 256), 256, 0, st>>>(g, a.gw, w.f0);
    k_gal_gather2<Real, R, true><<<cdiv(n, 256), 256, 0, st>>>(g, w.f0, nullptr, nullptr, a.gb,
                                                               a.gdb, w.ksc);
    k_kron_scalevec<Real><<<cdiv(n, 256), 256, 0, st>>>(g.nb, w.dg, w.ksc);
    k_zero<Real><<<cdiv(mp2, 256), 256, 0, st>>>(mp2, w.kt0);
    k_pcg_init<Real><<<cdiv(n, 256), 256, 0, st>>>(g.nb, w.mgp, w.f, nullptr, w.ksc, a.x, w.r,
                                                   w.z, w.p, w.kt0);
    kron_products<Real>(w, nullptr, st);
    k_kron_out_dot<Real><<<kDotBlocks, 256, 0, st>>>(g.nb, w.mgp, w.kt2, w.ksc, w.r, w.z, w.part2,
                                                     nullptr);
    k_dot2_fin<<<1, 256, 0, st>>>(w.part2, kDotBlocks, w.sc, 0, 4);  // r.z, F.F (r = F)
  } else {
    k_pcg_init<Real><<<cdiv(n, 256), 256, 0, st>>>(g.nb, 0, w.f, w.dg, nullptr, a.x, w.r, w.z,
                                                   w.p, nullptr);
    k_dot2_part<Real><<<kDotBlocks, 256, 0, st>>>(n, w.r, w.z, w.f, w.f, w.part2);
    k_dot2_fin<<<1, 256, 0, st>>>(w.part2, kDotBlocks, w.sc, 0, 4);
  }
}

// iters CG iterations; iteration it stores its r.z in slot it & 1 and its
// direction in p (it even) or p2 (it odd), reading the previous ones from the
// other slot and array.  Launches per iteration: operator, update, and with
// the Kronecker preconditioner 4 products and the scatter with the pairs
template <typename Real, int R>
static void gal_iters(const Geom& g, const GalerkinArgs<Real>& a, int iters, hipStream_t st) {
  constexpr int TC = gal_tc<Real, R>();
  const GalerkinWork<Real>& w = a.ws;
  const int ntx = cdiv(g.nb - 2, TC);  // tiles of interior coefficients per axis
  const int ntiles = ntx * ntx;
  const int nblk = 8 * cdiv(ntiles, 8);
  for (int it = 0; it < iters; ++it) {
    const int s_cur = it & 1, s_prev = s_cur ^ 1;
    Real* p_cur = s_cur ? w.p2 : w.p;
    const Real* p_prev = s_cur ? w.p : w.p2;
    k_gal_apply2<Real, R, TC><<<nblk, TC * TC, 0, st>>>(g, w.z, p_prev, p_cur, w.c, a.gb, a.gdb,
                                                        w.ap, w.part, w.part2, w.sc, s_cur,
                                                        s_prev, ntx, ntiles);
    if (a.precond == 1) {
      k_pcg_step1<Real, false><<<kDotBlocks, 256, 0, st>>>(g.nb, w.mgp, w.sc, s_cur, w.part,
                                                           ntiles, a.x, w.r, w.z, p_cur, w.ap,
                                                           w.dg, w.ksc, w.kt0, w.part2);
      kron_products<Real>(w, w.sc, st);
      k_kron_out_dot<Real><<<kDotBlocks, 256, 0, st>>>(g.nb, w.mgp, w.kt2, w.ksc, w.r, w.z,
                                                       w.part2, w.sc);
    } else {
      k_pcg_step1<Real, true><<<kDotBlocks, 256, 0, st>>>(g.nb, 0, w.sc, s_cur, w.part, ntiles,
                                                          a.x, w.r, w.z, p_cur, w.ap, w.dg,
                                                          nullptr, nullptr, w.part2);
    }
  }
}

template <typename Real>
void launch_galerkin_finish(const GalerkinWork<Real>& w, hipStream_t st) {
  k_dot2_fin<<<1, 256, 0, st>>>(w.part2, kDotBlocks, w.sc, 2, 3);
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
template void launch_galerkin_finish<float>(const GalerkinWork<float>&, hipStream_t);
template void launch_galerkin_finish<double>(const GalerkinWork<double>&, hipStream_t);

}  // namespace crv
