// Directional banded solves and the dense products of the Gram solve.
//
// The 1D factors are L D L^T with unit lower L of bandwidth r, computed in
// float64 once (eq. 14 for the B-spline mass matrix; eq. 28 for the shifted
// tridiagonal lines of the Gram matrix) and applied here in the working
// precision.
//
// Contiguous lines: one wavefront per line.  Lane l owns P consecutive
// entries.  Forward substitution is the order-r linear recurrence
//   y_j = b_j - sum_t L(j, j-t) y_{j-t},
// i.e. an affine map on the state (y_j, ..., y_{j-r+1}).  Each lane composes
// the maps of its chunk (a particular solution plus r homogeneous ones), a
// 6-step wavefront scan of the composed maps gives every lane its incoming
// state, and the lane re-runs its chunk from that state.  The backward sweep
// x_j = y_j / D_j - sum_t L(j+t, j) x_{j+t} is the same scan in reverse.
#include <algorithm>

#include "kernels.h"
#include <type_traits>

namespace crv {

template <typename Real, int R>
struct Affine {
  Real a[R][R];
  Real c[R];
};

template <typename Real, int R>
__device__ inline void compose(Affine<Real, R>& self, const Affine<Real, R>& prev) {
  // self <- self o prev : a = A_self A_prev, c = A_self c_prev + c_self
  Affine<Real, R> out;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    Real cc = self.c[i];
#pragma unroll
    for (int k = 0; k < R; ++k) cc += self.a[i][k] * prev.c[k];
    out.c[i] = cc;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      Real s = 0;
#pragma unroll
      for (int k = 0; k < R; ++k) s += self.a[i][k] * prev.a[k][j];
      out.a[i][j] = s;
    }
  }
  self = out;
}

template <typename Real, int R>
__device__ inline Affine<Real, R> shfl_affine(const Affine<Real, R>& v, int off, bool up) {
  Affine<Real, R> o;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    o.c[i] = up ? shfl_up(v.c[i], off) : shfl_down(v.c[i], off);
#pragma unroll
    for (int j = 0; j < R; ++j) o.a[i][j] = up ? shfl_up(v.a[i][j], off) : shfl_down(v.a[i][j], off);
  }
  return o;
}

// LDS index of entry j of a wave's line buffer, padded so the per-lane chunk
// reads (stride P) avoid bank conflicts.
template <int P>
__device__ inline int lidx(int j) {
  constexpr int S = (P % 2 == 0) ? P + 1 : P;
  return (j / P) * S + (j % P);
}

template <typename Real, int R, int P>
__global__ __launch_bounds__(256) void k_band_rows(const Real* __restrict__ b, Real* x, int n,
                                                   int nlines, int64_t line_stride,
                                                   const Real* __restrict__ lt,
                                                   const Real* __restrict__ invd, int64_t cs,
                                                   int64_t csd, int64_t zb) {
  b = zofs(b, zb); x = zofs(x, zb); lt = zofs(lt, zb); invd = zofs(invd, zb);
  constexpr int S = (P % 2 == 0) ? P + 1 : P;
  __shared__ Real buf[4][64 * S];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int line = blockIdx.x * 4 + w;
  const bool active = line < nlines;
  // an idle wave (past the last line) runs the scan on an empty line so the
  // block barriers stay uniform, and touches no memory
  n = active ? n : 0;
  const Real* bl = b + int64_t(line) * line_stride;
  Real* xl = x + int64_t(line) * line_stride;
  const Real* L = lt + int64_t(line) * cs;
  const Real* D = invd + int64_t(line) * csd;
  Real* sb = buf[w];
  if (active)
    for (int j = lane; j < n; j += 64) sb[lidx<P>(j)] = bl[j];
  __syncthreads();
  const int j0 = lane * P;
  Real v[P];
#pragma unroll
  for (int e = 0; e < P; ++e) v[e] = (j0 + e < n) ? sb[lane * S + e] : Real(0);
  // this lane's factor entries, all loaded before the recurrences use them
  // (forward: rows j0..j0+P-1; backward: up to R rows further; D^-1: own rows)
  Real lf[P + R][R], dd[P];
#pragma unroll
  for (int e = 0; e < P + R; ++e)
#pragma unroll
    for (int t = 0; t < R; ++t) lf[e][t] = (j0 + e < n) ? L[int64_t(j0 + e) * R + t] : Real(0);
#pragma unroll
  for (int e = 0; e < P; ++e) dd[e] = (j0 + e < n) ? D[j0 + e] : Real(0);

  // ---------------- forward: y_j = b_j - sum_t L(j,j-t) y_{j-t} --------------
  Affine<Real, R> f;
#pragma unroll
  for (int col = -1; col < R; ++col) {
    Real s[R];
#pragma unroll
    for (int t = 0; t < R; ++t) s[t] = (t == col) ? Real(1) : Real(0);
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int j = j0 + e;
      if (j < n) {
        Real y = (col < 0) ? v[e] : Real(0);
#pragma unroll
        for (int t = 1; t <= R; ++t) y -= lf[e][t - 1] * s[t - 1];
#pragma unroll
        for (int t = R - 1; t > 0; --t) s[t] = s[t - 1];
        s[0] = y;
      }
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
      if (col < 0) f.c[t] = s[t];
      else f.a[t][col] = s[t];
    }
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const Affine<Real, R> prev = shfl_affine(f, off, true);
    if (lane >= off) compose(f, prev);
  }
  {
    Real s[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const Real in = shfl_up(f.c[t], 1);
      s[t] = lane > 0 ? in : Real(0);
    }
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int j = j0 + e;
      if (j < n) {
        Real y = v[e];
#pragma unroll
        for (int t = 1; t <= R; ++t) y -= lf[e][t - 1] * s[t - 1];
#pragma unroll
        for (int t = R - 1; t > 0; --t) s[t] = s[t - 1];
        s[0] = y;
        v[e] = y * dd[e];  // z_j = y_j / D_j
      }
    }
  }

  // ------- backward: x_j = z_j - sum_t L(j+t, j) x_{j+t}, from j = n-1 down -------
  Affine<Real, R> g;
#pragma unroll
  for (int col = -1; col < R; ++col) {
    Real s[R];
#pragma unroll
    for (int t = 0; t < R; ++t) s[t] = (t == col) ? Real(1) : Real(0);
#pragma unroll
    for (int e = P - 1; e >= 0; --e) {
      const int j = j0 + e;
      if (j < n) {
        Real xv = (col < 0) ? v[e] : Real(0);
#pragma unroll
        for (int t = 1; t <= R; ++t)
          if (j + t < n) xv -= lf[e + t][t - 1] * s[t - 1];
#pragma unroll
        for (int t = R - 1; t > 0; --t) s[t] = s[t - 1];
        s[0] = xv;
      }
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
      if (col < 0) g.c[t] = s[t];
      else g.a[t][col] = s[t];
    }
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const Affine<Real, R> nxt = shfl_affine(g, off, false);
    if (lane + off < 64) compose(g, nxt);
  }
  {
    Real s[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const Real in = shfl_down(g.c[t], 1);
      s[t] = lane < 63 ? in : Real(0);
    }
#pragma unroll
    for (int e = P - 1; e >= 0; --e) {
      const int j = j0 + e;
      if (j < n) {
        Real xv = v[e];
#pragma unroll
        for (int t = 1; t <= R; ++t)
          if (j + t < n) xv -= lf[e + t][t - 1] * s[t - 1];
#pragma unroll
        for (int t = R - 1; t > 0; --t) s[t] = s[t - 1];
        s[0] = xv;
        v[e] = xv;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < P; ++e) sb[lane * S + e] = v[e];
  __syncthreads();
  if (active)
    for (int j = lane; j < n; j += 64) xl[j] = sb[lidx<P>(j)];
}

template <typename Real, int R>
static void band_rows_dispatch(int P, const Real* b, Real* x, int n, int nlines, int64_t ls,
                               const Real* lt, const Real* invd, int64_t cs, int64_t csd,
                               hipStream_t st, Batch bz) {
  dim3 grid(cdiv(nlines, 4), 1, bz.n);
#define CRV_P(PP) \
  case PP: k_band_rows<Real, R, PP><<<grid, 256, 0, st>>>(b, x, n, nlines, ls, lt, invd, cs, csd, bz.zb); break;
  switch (P) {
    CRV_P(1) CRV_P(2) CRV_P(3) CRV_P(4) CRV_P(5) CRV_P(8) CRV_P(9) CRV_P(12) CRV_P(16) CRV_P(17)
    default: break;
  }
#undef CRV_P
}

static int pick_p(int n) {
  static const int ps[] = {1, 2, 3, 4, 5, 8, 9, 12, 16, 17};
  for (int p : ps)
    if (64 * p >= n) return p;
  return -1;
}

// Tridiagonal contiguous lines (r = 1) without LDS: lane l reads its P
// entries of b, L and 1/D straight from memory (16-byte loads when the
// pitches allow), composes its chunk's map y -> a y + c, a 6-step shuffle
// scan gives it the incoming y, and the backward sweep
// x_j = y_j / D_j - L(j+1, j) x_{j+1} repeats this from the far end.
template <typename Real, int P>
__device__ inline void load_chunk(const Real* __restrict__ src, int j0, int n, bool vec, Real (&v)[P]) {
  constexpr int V = 16 / sizeof(Real);
  if constexpr (P % V == 0) {
    if (vec) {
      typedef Real vec_t __attribute__((ext_vector_type(V)));
#pragma unroll
      for (int e = 0; e < P; e += V) {
        const vec_t w = *reinterpret_cast<const vec_t*>(src + j0 + e);
#pragma unroll
        for (int k = 0; k < V; ++k) v[e + k] = w[k];
      }
#pragma unroll
      for (int e = 0; e < P; ++e)
        if (j0 + e >= n) v[e] = Real(0);
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < P; ++e) v[e] = (j0 + e < n) ? src[j0 + e] : Real(0);
}

template <typename Real, int P>
__global__ __launch_bounds__(256) void k_tridiag_rows(const Real* __restrict__ b,
                                                      Real* __restrict__ x, int n, int nlines,
                                                      int64_t ls, const Real* __restrict__ lt,
                                                      const Real* __restrict__ invd, int64_t cs,
                                                      int64_t csd, bool vec, int64_t zb) {
  b = zofs(b, zb); x = zofs(x, zb); lt = zofs(lt, zb); invd = zofs(invd, zb);
  const int lane = threadIdx.x & 63;
  const int line = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (line >= nlines) return;  // the wave leaves as a whole; no block barriers here
  const int j0 = lane * P;
  Real v[P], l[P], d[P];
  load_chunk<Real, P>(b + int64_t(line) * ls, j0, n, vec, v);
  load_chunk<Real, P>(lt + int64_t(line) * cs, j0, n, vec, l);
  load_chunk<Real, P>(invd + int64_t(line) * csd, j0, n, vec, d);
  // forward: y_j = b_j - l_j y_{j-1}; chunk map y_out = a y_in + c
  Real a = 1, c = 0;
#pragma unroll
  for (int e = 0; e < P; ++e)
    if (j0 + e < n) {
      c = v[e] - l[e] * c;
      a = -l[e] * a;
    }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const Real pa = shfl_up(a, off), pc = shfl_up(c, off);
    if (lane >= off) {
      c = a * pc + c;
      a = a * pa;
    }
  }
  Real y = shfl_up(c, 1);
  if (lane == 0) y = 0;
#pragma unroll
  for (int e = 0; e < P; ++e)
    if (j0 + e < n) {
      y = v[e] - l[e] * y;
      v[e] = y * d[e];  // z_j
    }
  // backward: x_j = z_j - l_{j+1} x_{j+1}; l_{j+1} of the last entry is the next lane's first
  Real lnext = shfl_down(l[0], 1);
  if (lane == 63) lnext = 0;
  a = 1;
  c = 0;
#pragma unroll
  for (int e = P - 1; e >= 0; --e)
    if (j0 + e < n) {
      const Real le = (e == P - 1) ? lnext : l[e + 1];
      c = v[e] - le * c;
      a = -le * a;
    }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const Real na = shfl_down(a, off), nc = shfl_down(c, off);
    if (lane + off < 64) {
      c = a * nc + c;
      a = a * na;
    }
  }
  Real xv = shfl_down(c, 1);
  if (lane == 63) xv = 0;
  Real* xl = x + int64_t(line) * ls;
#pragma unroll
  for (int e = P - 1; e >= 0; --e)
    if (j0 + e < n) {
      const Real le = (e == P - 1) ? lnext : l[e + 1];
      xv = v[e] - le * xv;
      v[e] = xv;
    }
  // the lane's P results leave as 16-byte stores when the loads could be
  // vectorised (then the whole span lies inside the line's pitch, and the
  // entries past n are the zeros the padded line holds)
  constexpr int V = 16 / sizeof(Real);
  if constexpr (P % V == 0) {
    if (vec) {
      typedef Real vec_t __attribute__((ext_vector_type(V)));
#pragma unroll
      for (int e = 0; e < P; e += V) {
        vec_t w;
#pragma unroll
        for (int k = 0; k < V; ++k) w[k] = v[e + k];
        *reinterpret_cast<vec_t*>(xl + j0 + e) = w;
      }
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < P; ++e)
    if (j0 + e < n) xl[j0 + e] = v[e];
}

template <typename Real>
void launch_band_rows(const Real* b, Real* x, int n, int nlines, int64_t line_stride, int r,
                      const Real* lt, const Real* inv_d, int64_t coef_stride,
                      int64_t coef_stride_d, hipStream_t st, Batch bz) {
  const int P = pick_p(n);
  if (P < 0 || nlines <= 0) return;
  if (r == 1 && coef_stride > 0 && coef_stride_d > 0) {
    // 16-byte loads need every lane's P entries inside each line's pitch and
    // 16-byte aligned line starts
    const int64_t V = 16 / int64_t(sizeof(Real));
    const int64_t span = 64 * int64_t(P);
    const bool vec = line_stride % V == 0 && coef_stride % V == 0 && coef_stride_d % V == 0 &&
                     span <= line_stride && span <= coef_stride && span <= coef_stride_d &&
                     reinterpret_cast<uintptr_t>(b) % 16 == 0 && reinterpret_cast<uintptr_t>(lt) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(inv_d) % 16 == 0;
    dim3 grid(cdiv(nlines, 4), 1, bz.n);
#define CRV_T(PP) \
  case PP: k_tridiag_rows<Real, PP><<<grid, 256, 0, st>>>(b, x, n, nlines, line_stride, lt, inv_d, coef_stride, coef_stride_d, vec, bz.zb); return;
    switch (P) {
      CRV_T(1) CRV_T(2) CRV_T(3) CRV_T(4) CRV_T(5) CRV_T(8) CRV_T(9) CRV_T(12) CRV_T(16) CRV_T(17)
      default: break;
    }
#undef CRV_T
  }
  switch (r) {
    case 1: band_rows_dispatch<Real, 1>(P, b, x, n, nlines, line_stride, lt, inv_d, coef_stride, coef_stride_d, st, bz); break;
    case 2: band_rows_dispatch<Real, 2>(P, b, x, n, nlines, line_stride, lt, inv_d, coef_stride, coef_stride_d, st, bz); break;
    default: band_rows_dispatch<Real, 3>(P, b, x, n, nlines, line_stride, lt, inv_d, coef_stride, coef_stride_d, st, bz); break;
  }
}

// Strided lines (element j of line c at x[j*row_stride + c]), shared
// coefficients.  A block owns 16 consecutive lines and splits their length
// into 64 chunks of at most CH rows: wave w, lane group s = lane/16 takes
// chunk 4w + s of line lane%16 (so a row access reads 4 runs of 16
// consecutive values).  The chunk's right-hand side is loaded once into
// registers (all of its rows in flight together) and stays there through
// both sweeps; the shared factors are staged in LDS.  Each chunk composes its
// affine map (particular solution + r homogeneous ones), 16 lanes of wave 0
// chain the 64 chunk maps of their line through LDS in order, and every chunk
// re-runs from its incoming state; the backward sweep repeats this from the
// far end, and the solution is stored once.
template <typename Real, int R, int CH>
__global__ __launch_bounds__(1024) void k_band_cols_scan(const Real* b, Real* x, int n,
                                                         int ncols, int64_t rs,
                                                         const Real* __restrict__ lt,
                                                         const Real* __restrict__ invd,
                                                         int64_t batch_stride) {
  constexpr int NCH = 64, CW = 16;  // chunks per line, lines per block
  constexpr int NM = R * R + R;      // one affine map
  constexpr int NMAX = NCH * CH;     // longest line
  __shared__ Real maps[NCH][NM][CW];
  __shared__ Real instate[NCH][R][CW];
  __shared__ Real slt[NMAX * R];
  __shared__ Real sinv[NMAX];
  const int tid = threadIdx.x;
  for (int k = tid; k < n * R; k += 1024) slt[k] = lt[k];
  for (int k = tid; k < n; k += 1024) sinv[k] = invd[k];
  const int lane = tid & 63, w = tid >> 6;
  const int cl = lane & (CW - 1), kc = w * 4 + (lane >> 4);  // line in block, chunk
  const int c = blockIdx.x * CW + cl;
  const bool colok = c < ncols;
  const int ch = (n + NCH - 1) / NCH;        // rows per chunk (<= CH)
  const int j0 = min(n, kc * ch), j1 = min(n, j0 + ch);
  const int len = j1 - j0;
  const Real* bb = b + int64_t(blockIdx.y) * batch_stride + (colok ? c : 0);
  Real* xx = x + int64_t(blockIdx.y) * batch_stride + (colok ? c : 0);
  Real v[CH];  // right-hand side, then z = D^-1 L^-1 b, then the solution
#pragma unroll
  for (int e = 0; e < CH; ++e) v[e] = (colok && e < len) ? bb[int64_t(j0 + e) * rs] : Real(0);
  __syncthreads();  // factors staged

  auto put_map = [&](const Real (&a)[R][R], const Real (&cc)[R]) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      maps[kc][R * R + i][cl] = cc[i];
#pragma unroll
      for (int k = 0; k < R; ++k) maps[kc][i * R + k][cl] = a[i][k];
    }
  };
  // the chunk's affine map of the forward recurrence y_j = v_j - sum_t l_jt y_(j-t)
  auto forward_map = [&]() {
    Real a[R][R], cc[R];
#pragma unroll
    for (int col = -1; col < R; ++col) {
      Real st[R];
#pragma unroll
      for (int t = 0; t < R; ++t) st[t] = (t == col) ? Real(1) : Real(0);
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        if (e < len) {
          const int j = j0 + e;
          Real y = (col < 0) ? v[e] : Real(0);
#pragma unroll
          for (int t = 1; t <= R; ++t) y -= slt[j * R + (t - 1)] * st[t - 1];
#pragma unroll
          for (int t = R - 1; t > 0; --t) st[t] = st[t - 1];
          st[0] = y;
        }
      }
#pragma unroll
      for (int t = 0; t < R; ++t) {
        if (col < 0) cc[t] = st[t];
        else a[t][col] = st[t];
      }
    }
    put_map(a, cc);
  };
  // the same for the backward recurrence x_j = z_j - sum_t l_(j+t)t x_(j+t),
  // taken from the chunk's last row to its first
  auto backward_map = [&]() {
    Real a[R][R], cc[R];
#pragma unroll
    for (int col = -1; col < R; ++col) {
      Real st[R];
#pragma unroll
      for (int t = 0; t < R; ++t) st[t] = (t == col) ? Real(1) : Real(0);
#pragma unroll
      for (int e = CH - 1; e >= 0; --e) {
        if (e < len) {
          const int j = j0 + e;
          Real y = (col < 0) ? v[e] : Real(0);
#pragma unroll
          for (int t = 1; t <= R; ++t)
            if (j + t < n) y -= slt[(j + t) * R + (t - 1)] * st[t - 1];
#pragma unroll
          for (int t = R - 1; t > 0; --t) st[t] = st[t - 1];
          st[0] = y;
        }
      }
#pragma unroll
      for (int t = 0; t < R; ++t) {
        if (col < 0) cc[t] = st[t];
        else a[t][col] = st[t];
      }
    }
    put_map(a, cc);
  };
  // lanes 0..15 of wave 0 chain their line's chunk maps in order (dir 0:
  // first to last chunk)
  auto scan = [&](int dir) {
    if (w != 0 || lane >= CW) return;
    Real st[R];
#pragma unroll
    for (int t = 0; t < R; ++t) st[t] = 0;
    for (int k = 0; k < NCH; ++k) {
      const int q = dir == 0 ? k : NCH - 1 - k;
#pragma unroll
      for (int t = 0; t < R; ++t) instate[q][t][cl] = st[t];
      Real nx[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        Real acc = maps[q][R * R + i][cl];
#pragma unroll
        for (int k2 = 0; k2 < R; ++k2) acc += maps[q][i * R + k2][cl] * st[k2];
        nx[i] = acc;
      }
#pragma unroll
      for (int t = 0; t < R; ++t) st[t] = nx[t];
    }
  };

  if (colok) forward_map();
  __syncthreads();
  scan(0);
  __syncthreads();
  if (colok) {
    Real st[R];
#pragma unroll
    for (int t = 0; t < R; ++t) st[t] = instate[kc][t][cl];
#pragma unroll
    for (int e = 0; e < CH; ++e) {
      if (e < len) {
        const int j = j0 + e;
        Real y = v[e];
#pragma unroll
        for (int t = 1; t <= R; ++t) y -= slt[j * R + (t - 1)] * st[t - 1];
#pragma unroll
        for (int t = R - 1; t > 0; --t) st[t] = st[t - 1];
        st[0] = y;
        v[e] = y * sinv[j];  // z_j = y_j / D_j
      }
    }
  }
  __syncthreads();  // the forward scan's maps and states are read before they are replaced
  if (colok) backward_map();
  __syncthreads();
  scan(1);
  __syncthreads();
  if (colok) {
    Real st[R];
#pragma unroll
    for (int t = 0; t < R; ++t) st[t] = instate[kc][t][cl];
#pragma unroll
    for (int e = CH - 1; e >= 0; --e) {
      if (e < len) {
        const int j = j0 + e;
        Real xv = v[e];
#pragma unroll
        for (int t = 1; t <= R; ++t)
          if (j + t < n) xv -= slt[(j + t) * R + (t - 1)] * st[t - 1];
#pragma unroll
        for (int t = R - 1; t > 0; --t) st[t] = st[t - 1];
        st[0] = xv;
        v[e] = xv;
      }
    }
#pragma unroll
    for (int e = 0; e < CH; ++e)
      if (e < len) xx[int64_t(j0 + e) * rs] = v[e];
  }
}

template <typename Real, int R>
static void band_cols_dispatch(const Real* b, Real* x, int n, int nlines, int64_t rs,
                               const Real* lt, const Real* inv_d, int64_t batch,
                               int64_t batch_stride, hipStream_t st) {
  dim3 grid(cdiv(nlines, 16), unsigned(batch));
  const int ch = cdiv(n, 64);
  // lines are n = n_elem + degree <= 1027 long (at most 17 rows per chunk)
  if (ch <= 5)
    k_band_cols_scan<Real, R, 5><<<grid, 1024, 0, st>>>(b, x, n, nlines, rs, lt, inv_d, batch_stride);
  else if (ch <= 9)
    k_band_cols_scan<Real, R, 9><<<grid, 1024, 0, st>>>(b, x, n, nlines, rs, lt, inv_d, batch_stride);
  else if (ch <= 17)
    k_band_cols_scan<Real, R, 17><<<grid, 1024, 0, st>>>(b, x, n, nlines, rs, lt, inv_d, batch_stride);
}

template <typename Real>
void launch_band_cols(const Real* b, Real* x, int n, int nlines, int64_t row_stride, int r,
                      const Real* lt, const Real* inv_d, int64_t batch, int64_t batch_stride,
                      hipStream_t st, Batch bz) {
  if (nlines <= 0) return;
  if (bz.n > 1) {
    // scenarios of a batch are the planes of the launch (2D passes have one
    // plane); the factors are the same table in every scenario's workspace
    if (batch != 1) return;
    batch = bz.n;
    batch_stride = bz.zb / int64_t(sizeof(Real));
  }
  switch (r) {
    case 1: band_cols_dispatch<Real, 1>(b, x, n, nlines, row_stride, lt, inv_d, batch, batch_stride, st); break;
    case 2: band_cols_dispatch<Real, 2>(b, x, n, nlines, row_stride, lt, inv_d, batch, batch_stride, st); break;
    default: band_cols_dispatch<Real, 3>(b, x, n, nlines, row_stride, lt, inv_d, batch, batch_stride, st); break;
  }
}

// ---------------------------------------------------------------------------
// C = A B (row-major, dims multiples of 64): 64x64 tiles, 16-deep K slabs in
// LDS, 4x4 outputs per thread.  blockIdx.z selects one product of a batch
// that shares A (B and C advance by sb and sc).
// ---------------------------------------------------------------------------
// EPI (this kernel and k_gemm_pa_f32): 0 stores C; 1 stores C^T (square C);
// 2 stores C_ij / (sym[M+i] sym[j] + sym[i] sym[M+j]) (square C; the
// Kronecker symbol of the Galerkin preconditioner).  skip (nullable): the
// whole product is left out when skip[0] <= skip[3] (an iterative solve's
// residual against its threshold, read from device memory)
template <typename Real, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const Real* __restrict__ A,
                                              int lda, const Real* __restrict__ B, int ldb,
                                              int64_t sb, Real* __restrict__ C, int ldc,
                                              int64_t sc, const Real* __restrict__ sym,
                                              const double* __restrict__ skip) {
  if (skip && skip[0] <= skip[3]) return;
  B += int64_t(blockIdx.z) * sb;
  C += int64_t(blockIdx.z) * sc;
  __shared__ Real As[16][64 + 4];
  __shared__ Real Bs[16][64 + 4];
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  Real acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    {
      const int mm = tid / 4, kk = (tid % 4) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) As[kk + q][mm] = A[int64_t(m0 + mm) * lda + k0 + kk + q];
      const int kb = tid / 16, nn = (tid % 16) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) Bs[kb][nn + q] = B[int64_t(k0 + kb) * ldb + n0 + nn + q];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      Real a[4], bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[k][ty * 4 + q];
        bv[q] = Bs[k][tx * 4 + q];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * bv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gi = m0 + ty * 4 + i, gj = n0 + tx * 4 + j;
      if constexpr (EPI == 1) {
        C[int64_t(gj) * ldc + gi] = acc[i][j];
      } else if constexpr (EPI == 2) {
        C[int64_t(gi) * ldc + gj] = acc[i][j] / (sym[M + gi] * sym[gj] + sym[gi] * sym[M + gj]);
      } else {
        C[int64_t(gi) * ldc + gj] = acc[i][j];
      }
    }
}

// float32 C = A B on the matrix cores (v_mfma_f32_32x32x2f32): one 32x32
// output tile per block; the 4 waves split K in four contiguous ranges and
// their partial tiles are summed in a fixed order through LDS.  Lane
// (r = lane%32, g = lane/32) feeds A[m0+r][k+g] and B[k+g][n0+r] per step.
typedef float gemm_f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gemm_mfma_f32(int M, int N, int K,
                                                       const float* __restrict__ A, int lda,
                                                       const float* __restrict__ B, int ldb,
                                                       int64_t sb, float* __restrict__ C, int ldc,
                                                       int64_t sc) {
  B += int64_t(blockIdx.z) * sb;
  C += int64_t(blockIdx.z) * sc;
  __shared__ float part[4][32 * 33];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 31, g = lane >> 5;
  const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
  const int kq = K / 4, kb = w * kq;
  const float* a = A + int64_t(m0 + r) * lda + kb + g;
  const float* b = B + int64_t(kb + g) * ldb + n0 + r;
  gemm_f32x16_t acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (int k = 0; k < kq; k += 16) {
    float av[8], bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      av[u] = a[k + 2 * u];
      bv[u] = b[int64_t(k + 2 * u) * ldb];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u], bv[u], acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) part[w][(8 * (i >> 2) + 4 * g + (i & 3)) * 33 + r] = acc[i];
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += 256) {
    const int row = e >> 5, col = e & 31;
    const float v = ((part[0][row * 33 + col] + part[1][row * 33 + col]) + part[2][row * 33 + col]) +
                    part[3][row * 33 + col];
    C[int64_t(m0 + row) * ldc + n0 + col] = v;
  }
}

// float32 C = A B with A supplied as packed 32x32x2 fragments (A is a
// constant operand, packed once): chunk kc of row block mb holds, for lane
// (r = lane%32, g = lane/32), A[32 mb + r][16 kc + 2u + g], u = 0..7, as 8
// consecutive floats, so every A load of a wave is one contiguous 2 KB read.
// One 32x32 output tile per block; K is split into NW * RPW contiguous
// ranges, RPW per wave, and the range sums are combined in a fixed order
// (through registers within a wave, through LDS across waves).
template <int EPI, int NW, int RPW>
__global__ __launch_bounds__(64 * NW) void k_gemm_pa_f32(int M, int N, int K,
                                                         const float* __restrict__ Af,
                                                         const float* __restrict__ B, int ldb,
                                                         int64_t sb, float* __restrict__ C, int ldc,
                                                         int64_t sc, const float* __restrict__ sym,
                                                         const double* __restrict__ skip) {
  if (skip && skip[0] <= skip[3]) return;
  B += int64_t(blockIdx.z) * sb;
  C += int64_t(blockIdx.z) * sc;
  // K ranges: wave w sums ranges RPW w .. RPW w + RPW - 1 (RPW = 1 or 2).  The
  // range sums combine as: adjacent pairs first (0+1, 2+3, ...), then the
  // pair sums in order (an odd range count: all ranges in order), the same
  // sum whether a pair is added in a wave's registers or from LDS
  constexpr int R = NW * RPW;
  __shared__ float part[NW][32 * 33];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 31, g = lane >> 5;
  const int mb = blockIdx.y, n0 = blockIdx.x * 32;
  const int kq = K / R;  // multiple of 16
  gemm_f32x16_t tot;
#pragma unroll
  for (int j = 0; j < RPW; ++j) {
    const int q = w * RPW + j;
    const float* a = Af + ((int64_t(mb) * (K / 16) + (q * kq) / 16) * 64 + lane) * 8;
    const float* b = B + int64_t(q * kq + g) * ldb + n0 + r;
    gemm_f32x16_t acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
    // 16-deep K chunks.  For the common chunk counts of single launches the
    // loop is unrolled and software-pipelined over two register sets: chunk kc + 1's loads are
    // issued before chunk kc's products (scheduling barriers keep them there;
    // left alone, the scheduler sinks the loads below the products).  The
    // products keep their order, so the sum is the same either way.
    const int nkc = kq / 16;
    auto load = [&](int kc, f32x4_t& x0, f32x4_t& x1, float (&y)[8]) {
      x0 = *reinterpret_cast<const f32x4_t*>(a + kc * 512);
      x1 = *reinterpret_cast<const f32x4_t*>(a + kc * 512 + 4);
#pragma unroll
      for (int u = 0; u < 8; ++u) y[u] = b[int64_t(kc * 16 + 2 * u) * ldb];
    };
    auto products = [&](const f32x4_t& x0, const f32x4_t& x1, const float (&y)[8]) {
      const float av[8] = {x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]};
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u], y[u], acc, 0, 0, 0);
    };
    auto pipelined = [&](auto nk) {
      constexpr int NK = decltype(nk)::value;
      f32x4_t x0[2], x1[2];
      float y[2][8];
      load(0, x0[0], x1[0], y[0]);
#pragma unroll
      for (int kc = 0; kc < NK; ++kc) {
        if (kc + 1 < NK) load(kc + 1, x0[(kc + 1) & 1], x1[(kc + 1) & 1], y[(kc + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        products(x0[kc & 1], x1[kc & 1], y[kc & 1]);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    // (one range per wave only: with two ranges per wave, as in batched
    // launches, the barriers cost more than the overlap gains: 8-scenario
    // product 34 -> 48 us)
    if (RPW == 1 && nkc == 4) {
      pipelined(std::integral_constant<int, 4>{});
    } else if (RPW == 1 && nkc == 8) {
      pipelined(std::integral_constant<int, 8>{});
    } else {
      for (int kc = 0; kc < nkc; ++kc) {
        f32x4_t x0, x1;
        float y[8];
        load(kc, x0, x1, y);
        products(x0, x1, y);
      }
    }
    if (j == 0) tot = acc;
    else tot += acc;  // the pair sum of ranges 2w, 2w + 1
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) part[w][(8 * (i >> 2) + 4 * g + (i & 3)) * 33 + r] = tot[i];
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += 64 * NW) {
    // the transposed store walks the tile by columns, so both stores are
    // contiguous along the lanes
    const int row = EPI == 1 ? (e & 31) : (e >> 5), col = EPI == 1 ? (e >> 5) : (e & 31);
    const int at = row * 33 + col;
    float v;
    if constexpr (RPW == 1 && R % 2 == 0) {
      v = part[0][at] + part[1][at];
      for (int k = 1; k < R / 2; ++k) v += part[2 * k][at] + part[2 * k + 1][at];
    } else {
      v = part[0][at];
      for (int k = 1; k < NW; ++k) v += part[k][at];
    }
    const int gi = mb * 32 + row, gj = n0 + col;
    if constexpr (EPI == 1) {
      C[int64_t(gj) * ldc + gi] = v;
    } else if constexpr (EPI == 2) {
      C[int64_t(gi) * ldc + gj] = v / (sym[M + gi] * sym[gj] + sym[gi] * sym[M + gj]);
    } else {
      C[int64_t(gi) * ldc + gj] = v;
    }
  }
}

template <typename Real, int EPI>
static void gemm_dispatch(int M, int N, int K, const Real* A, int lda, const Real* B, int ldb,
                          int64_t sb, Real* C, int ldc, int64_t sc, int batch, hipStream_t st,
                          const Real* a_packed, const Real* sym, const double* skip) {
  if (batch <= 0) return;
  if constexpr (sizeof(Real) == 4) {
    if (EPI != 0 || a_packed) {  // epilogues: callers always pass the packed operand
      // K split into nr ranges (the largest divisor of K/64 up to 8), so that
      // every range is a multiple of 16.  One wave per range, or two ranges
      // per wave once the grid has 512 or more tiles (as in batched launches:
      // blocks of half the waves and half the LDS run beside the other
      // streams' kernels better); the sums are the same either way
      const int units = K / 64;
      int nr = 1;
      for (int d = 8; d >= 1; --d)
        if (units % d == 0) {
          nr = d;
          break;
        }
      const bool pairs = nr % 2 == 0 && int64_t(N / 32) * (M / 32) * batch >= 512;
      dim3 grid(N / 32, M / 32, batch);
#define CRV_PA(NWV, RPWV) \
  k_gemm_pa_f32<EPI, NWV, RPWV><<<grid, 64 * NWV, 0, st>>>(M, N, K, a_packed, B, ldb, sb, C, ldc, sc, sym, skip)
      if (pairs) {
        switch (nr / 2) {
          case 1: CRV_PA(1, 2); break;
          case 2: CRV_PA(2, 2); break;
          case 3: CRV_PA(3, 2); break;
          default: CRV_PA(4, 2); break;
        }
      } else {
        switch (nr) {
          case 1: CRV_PA(1, 1); break;
          case 2: CRV_PA(2, 1); break;
          case 3: CRV_PA(3, 1); break;
          case 4: CRV_PA(4, 1); break;
          case 5: CRV_PA(5, 1); break;
          case 6: CRV_PA(6, 1); break;
          case 7: CRV_PA(7, 1); break;
          default: CRV_PA(8, 1); break;
        }
      }
#undef CRV_PA
      return;
    }
    // dims are multiples of 64, so K/4 is a multiple of 16
    dim3 grid(N / 32, M / 32, batch);
    k_gemm_mfma_f32<<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, sb, C, ldc, sc);
  } else {
    dim3 grid(N / 64, M / 64, batch);
    k_gemm<Real, EPI><<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, sb, C, ldc, sc, sym, skip);
  }
}

template <typename Real>
void launch_gemm_batched(int M, int N, int K, const Real* A, int lda, const Real* B, int ldb,
                         int64_t sb, Real* C, int ldc, int64_t sc, int batch, hipStream_t st,
                         const Real* a_packed) {
  gemm_dispatch<Real, 0>(M, N, K, A, lda, B, ldb, sb, C, ldc, sc, batch, st, a_packed, nullptr,
                         nullptr);
}

template <typename Real>
void launch_gemm_sq_epi(int M, const Real* A, const Real* B, Real* C, int epi, const Real* sym,
                        hipStream_t st, const Real* a_packed, const double* skip) {
  if (sizeof(Real) == 4 && !a_packed) return;  // float epilogues run on the packed kernel only
  if (epi == 1)
    gemm_dispatch<Real, 1>(M, M, M, A, M, B, M, 0, C, M, 0, 1, st, a_packed, sym, skip);
  else if (epi == 2)
    gemm_dispatch<Real, 2>(M, M, M, A, M, B, M, 0, C, M, 0, 1, st, a_packed, sym, skip);
  else
    gemm_dispatch<Real, 0>(M, M, M, A, M, B, M, 0, C, M, 0, 1, st, a_packed, sym, skip);
}

template <typename Real>
void launch_gemm(int M, int N, int K, const Real* A, int lda, const Real* B, int ldb, Real* C,
                 int ldc, hipStream_t st, const Real* a_packed) {
  launch_gemm_batched<Real>(M, N, K, A, lda, B, ldb, 0, C, ldc, 0, 1, st, a_packed);
}

#define CRV_INST(R)                                                                            \
  template void launch_band_rows<R>(const R*, R*, int, int, int64_t, int, const R*, const R*, \
                                    int64_t, int64_t, hipStream_t, Batch);                    \
  template void launch_band_cols<R>(const R*, R*, int, int, int64_t, int, const R*, const R*, \
                                    int64_t, int64_t, hipStream_t, Batch);                    \
  template void launch_gemm<R>(int, int, int, const R*, int, const R*, int, R*, int, hipStream_t, \
                               const R*);                                                     \
  template void launch_gemm_batched<R>(int, int, int, const R*, int, const R*, int, int64_t, R*, \
                                       int, int64_t, int, hipStream_t, const R*);                \
  template void launch_gemm_sq_epi<R>(int, const R*, const R*, R*, int, const R*, hipStream_t,  \
                                      const R*, const double*);
CRV_INST(float)
CRV_INST(double)

}  // namespace crv
