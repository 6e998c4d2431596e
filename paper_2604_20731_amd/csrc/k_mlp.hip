// Pressure network u = m NN_theta(2x - 1) on the collocation nodes: forward,
// backward with per-layer recomputation, fixed-order gradient reduction and
// the fused Adam update.
//
// This file holds the per-node (one thread per node) formulation used for
// float64 verification runs and small grids; the matrix-core formulation for
// float32 and bf16 lives in k_mlp_mfma.hip.
//
// Parameter layout: per layer W (out x in, row-major) then b; layers
// d -> width (tanh) -> ... -> width (tanh) -> 1 (linear).
#include "kernels.h"

namespace crv {

int64_t mlp_param_count(int dim, int width, int hidden) {
  int64_t p = int64_t(width) * dim + width;
  p += int64_t(hidden - 1) * (int64_t(width) * width + width);
  p += width + 1;
  return p;
}

template <typename Real, int DIM>
__device__ inline void node_input(const Geom& g, int64_t p, Real* z, bool* interior, Real* fac) {
  const int n = g.n;
  const int i = int(p % n);
  const int j = int((p / n) % n);
  const int k = DIM == 3 ? int(p / (int64_t(n) * n)) : 0;
  const double inv = 1.0 / double(g.ne);
  z[0] = Real(2.0 * (double(i) * inv) - 1.0);
  z[1] = Real(2.0 * (double(j) * inv) - 1.0);
  if (DIM == 3) z[2 % DIM] = Real(2.0 * (double(k) * inv) - 1.0);
  bool in = i > 0 && i < g.ne && j > 0 && j < g.ne;
  if (DIM == 3) in = in && k > 0 && k < g.ne;
  *interior = in;
  *fac = in ? Real(trial_factor<DIM>(g.bfac, g.ne, i, j, k)) : Real(0);
}

// exact i/N as the oracle computes it (double division, then scaling)
template <typename Real, int W, int DIM>
__global__ __launch_bounds__(256) void k_mlp_fwd(Geom g, int hidden, const Real* __restrict__ th,
                                                 Real* __restrict__ u, long long* t_bump) {
  const int64_t total = ipow(g.n, DIM);
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t_bump && p == 0) *t_bump = *t_bump + 1;  // first kernel of an Adam iteration
  if (p >= total) return;
  Real z[DIM], fac;
  bool interior;
  node_input<Real, DIM>(g, p, z, &interior, &fac);
  Real h[W], hn[W];
  const Real* w = th;
#pragma unroll
  for (int o = 0; o < W; ++o) {
    Real a = w[W * DIM + o];
#pragma unroll
    for (int c = 0; c < DIM; ++c) a += w[o * DIM + c] * z[c];
    h[o] = tanh_fast(a);
  }
  w += W * DIM + W;
  for (int l = 1; l < hidden; ++l) {
#pragma unroll
    for (int o = 0; o < W; ++o) {
      Real a = w[W * W + o];
#pragma unroll
      for (int i = 0; i < W; ++i) a += w[o * W + i] * h[i];
      hn[o] = tanh_fast(a);
    }
#pragma unroll
    for (int o = 0; o < W; ++o) h[o] = hn[o];
    w += W * W + W;
  }
  Real y = w[W];
#pragma unroll
  for (int i = 0; i < W; ++i) y += w[i] * h[i];
  u[p] = interior ? fac * y : Real(0);
}

// Backward: a block of NT threads handles NT nodes per tile and loops over
// tiles; it recomputes the forward pass (hidden activations kept in LDS,
// layer by layer), back-propagates g_u, and accumulates the parameter
// gradient of its tiles into its own row of `partials` in a fixed order.
template <typename Real, int W, int DIM>
__global__ __launch_bounds__(256) void k_mlp_bwd(Geom g, int hidden, int64_t P,
                                                 const Real* __restrict__ th,
                                                 const Real* __restrict__ gu,
                                                 Real* __restrict__ partials) {
  extern __shared__ unsigned char smem_raw[];
  Real* smem = reinterpret_cast<Real*>(smem_raw);
  const int NT = blockDim.x;
  const int tid = threadIdx.x;
  Real* Hs = smem;                               // hidden x W x NT
  Real* Ds = Hs + int64_t(hidden) * W * NT;      // W x NT
  Real* Zs = Ds + W * NT;                        // DIM x NT
  Real* Gs = Zs + DIM * NT;                      // NT
  Real* row = partials + int64_t(blockIdx.x) * P;
  for (int64_t q = tid; q < P; q += NT) row[q] = Real(0);
  const int64_t total = ipow(g.n, DIM);
  const int64_t ntiles = (total + NT - 1) / NT;
  const int64_t off_out = int64_t(W) * DIM + W + int64_t(hidden - 1) * (int64_t(W) * W + W);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t p = tile * NT + tid;
    const bool valid = p < total;
    Real z[DIM], fac = 0;
    bool interior = false;
    if (valid) node_input<Real, DIM>(g, p, z, &interior, &fac);
    else
      for (int c = 0; c < DIM; ++c) z[c] = 0;
    for (int c = 0; c < DIM; ++c) Zs[c * NT + tid] = z[c];
    // forward, storing every hidden activation
    Real h[W], hn[W];
    {
      const Real* w = th;
#pragma unroll
      for (int o = 0; o < W; ++o) {
        Real a = w[W * DIM + o];
#pragma unroll
        for (int c = 0; c < DIM; ++c) a += w[o * DIM + c] * z[c];
        h[o] = tanh_fast(a);
        Hs[o * NT + tid] = h[o];
      }
      w += W * DIM + W;
      for (int l = 1; l < hidden; ++l) {
#pragma unroll
        for (int o = 0; o < W; ++o) {
          Real a = w[W * W + o];
#pragma unroll
          for (int i = 0; i < W; ++i) a += w[o * W + i] * h[i];
          hn[o] = tanh_fast(a);
        }
#pragma unroll
        for (int o = 0; o < W; ++o) {
          h[o] = hn[o];
          Hs[(int64_t(l) * W + o) * NT + tid] = h[o];
        }
        w += W * W + W;
      }
    }
    const Real gv = (valid && interior) ? fac * gu[p] : Real(0);  // dLOSS/dNN = f dLOSS/du
    Gs[tid] = gv;
    // delta of the last hidden layer: g * w_out * (1 - h^2)
    {
      const Real* wo = th + off_out;
#pragma unroll
      for (int i = 0; i < W; ++i) Ds[i * NT + tid] = gv * wo[i] * (Real(1) - h[i] * h[i]);
    }
    __syncthreads();
    // output layer gradient: dW_out[i] = sum_n g_n h_H[i][n], db_out = sum_n g_n
    {
      const Real* Hl = Hs + int64_t(hidden - 1) * W * NT;
      for (int i = tid; i <= W; i += NT) {
        Real s = 0;
        if (i < W)
          for (int nn = 0; nn < NT; ++nn) s += Gs[nn] * Hl[i * NT + nn];
        else
          for (int nn = 0; nn < NT; ++nn) s += Gs[nn];
        row[off_out + i] += s;
      }
    }
    for (int l = hidden; l >= 1; --l) {
      const int in_dim = (l == 1) ? DIM : W;
      const Real* In = (l == 1) ? Zs : Hs + int64_t(l - 2) * W * NT;
      const int64_t off = (l == 1) ? 0 : int64_t(W) * DIM + W + int64_t(l - 2) * (int64_t(W) * W + W);
      // dW_l[o][i] = sum_n D[o][n] In[i][n];  db_l[o] = sum_n D[o][n]
      for (int idx = tid; idx < W * (in_dim + 1); idx += NT) {
        const int o = idx / (in_dim + 1), i = idx % (in_dim + 1);
        Real s = 0;
        if (i < in_dim)
          for (int nn = 0; nn < NT; ++nn) s += Ds[o * NT + nn] * In[i * NT + nn];
        else
          for (int nn = 0; nn < NT; ++nn) s += Ds[o * NT + nn];
        if (i < in_dim) row[off + int64_t(o) * in_dim + i] += s;
        else row[off + int64_t(W) * in_dim + o] += s;
      }
      if (l > 1) {
        // delta_{l-1}[i] = (sum_o W_l[o][i] delta_l[o]) (1 - h_{l-1}[i]^2), own node only
        const Real* wl = th + off;
        Real dn[W];
#pragma unroll
        for (int i = 0; i < W; ++i) dn[i] = 0;
        for (int o = 0; o < W; ++o) {
          const Real d = Ds[o * NT + tid];
#pragma unroll
          for (int i = 0; i < W; ++i) dn[i] += wl[o * W + i] * d;
        }
        const Real* Hp = Hs + int64_t(l - 2) * W * NT;
        __syncthreads();  // every thread is done reading Ds
#pragma unroll
        for (int i = 0; i < W; ++i) {
          const Real hv = Hp[i * NT + tid];
          Ds[i * NT + tid] = dn[i] * (Real(1) - hv * hv);
        }
      }
      __syncthreads();
    }
  }
}

// threads (= nodes) per backward tile: the largest of 64/32/16/8 whose LDS
// (all hidden activations + one delta layer + inputs) stays within 64 KB
static int bwd_nt(int width, int hidden, int real_bytes) {
  for (int nt = 64; nt >= 8; nt /= 2) {
    const int64_t bytes = (int64_t(hidden) * width * nt + int64_t(width) * nt + 4 * nt) * real_bytes;
    if (bytes <= 64 * 1024) return nt;
  }
  return 8;
}

static int64_t bwd_lds(int width, int hidden, int dim, int nt, int real_bytes) {
  return (int64_t(hidden) * width * nt + int64_t(width) * nt + int64_t(dim) * nt + nt) * real_bytes;
}

constexpr int kMaxBwdBlocks = 1024;

int mlp_backward_rows(const Geom& g, const MlpShape& s, int real_bytes) {
  const int nt = bwd_nt(s.width, s.hidden, real_bytes);
  const int64_t total = ipow(g.n, s.dim);
  return int(std::min<int64_t>((total + nt - 1) / nt, kMaxBwdBlocks));
}

template <typename Real>
void launch_mlp_forward(const Geom& g, const MlpShape& s, const Real* theta, Real* u,
                        long long* t_bump, hipStream_t st) {
  const int64_t total = ipow(g.n, s.dim);
  dim3 grid(cdiv(total, 256));
#define CRV_F(WW, DD) \
  if (s.width == WW && s.dim == DD) { k_mlp_fwd<Real, WW, DD><<<grid, 256, 0, st>>>(g, s.hidden, theta, u, t_bump); return; }
  CRV_F(16, 2) CRV_F(32, 2) CRV_F(64, 2) CRV_F(128, 2)
  CRV_F(16, 3) CRV_F(32, 3) CRV_F(64, 3) CRV_F(128, 3)
#undef CRV_F
}

template <typename Real>
int launch_mlp_backward(const Geom& g, const MlpShape& s, const Real* theta, const Real* gu,
                        Real* partials, hipStream_t st) {
  const int nt = bwd_nt(s.width, s.hidden, sizeof(Real));
  const int rows = mlp_backward_rows(g, s, sizeof(Real));
  const size_t lds = size_t(bwd_lds(s.width, s.hidden, s.dim, nt, sizeof(Real)));
#define CRV_B(WW, DD)                                                                   \
  if (s.width == WW && s.dim == DD) {                                                   \
    k_mlp_bwd<Real, WW, DD><<<rows, nt, lds, st>>>(g, s.hidden, s.nparams, theta, gu, partials); \
    return rows;                                                                        \
  }
  CRV_B(16, 2) CRV_B(32, 2) CRV_B(64, 2) CRV_B(128, 2)
  CRV_B(16, 3) CRV_B(32, 3) CRV_B(64, 3) CRV_B(128, 3)
#undef CRV_B
  return rows;
}

// out[c][p] = sum_{r in chunk c} in[r][p], chunks of 64 rows, fixed order.
template <typename Real>
__global__ __launch_bounds__(256) void k_reduce_rows(const Real* __restrict__ in, int rows,
                                                     int64_t P, int64_t ld,
                                                     Real* __restrict__ out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int r0 = blockIdx.y * 64, r1 = min(rows, r0 + 64);
  Real s = 0;
  for (int r = r0; r < r1; ++r) s += in[int64_t(r) * ld + p];
  out[int64_t(blockIdx.y) * P + p] = s;
}

template <typename Real>
void launch_reduce_rows(const Real* in, int rows, int64_t P, int64_t ld, Real* scratch, Real* out,
                        hipStream_t st) {
  const Real* src = in;
  int64_t src_ld = ld;
  int nrows = rows;
  Real* bufs[2] = {scratch, scratch + int64_t(cdiv(rows, 64)) * P};
  int which = 0;
  while (true) {
    const int nout = cdiv(nrows, 64);
    Real* dst = (nout == 1) ? out : bufs[which];
    dim3 grid(cdiv(P, 256), nout);
    k_reduce_rows<Real><<<grid, 256, 0, st>>>(src, nrows, P, src_ld, dst);
    if (nout == 1) break;
    src = dst;
    src_ld = P;
    nrows = nout;
    which ^= 1;
  }
}

// Adam (t already counts this update): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
template <typename Real>
__global__ __launch_bounds__(256) void k_adam(int64_t P, Real* __restrict__ th, Real* __restrict__ m,
                                              Real* __restrict__ v, const Real* __restrict__ g,
                                              double lr, double b1, double b2, double eps,
                                              const long long* __restrict__ t_dev) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double t = double(*t_dev);
  const Real c1 = Real(1.0 - pow(b1, t)), c2 = Real(1.0 - pow(b2, t));
  const Real gg = g[p];
  const Real mm = Real(b1) * m[p] + Real(1.0 - b1) * gg;
  const Real vv = Real(b2) * v[p] + Real(1.0 - b2) * gg * gg;
  m[p] = mm;
  v[p] = vv;
  const Real mhat = mm / c1, vhat = vv / c2;
  th[p] = th[p] - Real(lr) * mhat / (sqrt(vhat) + Real(eps));
}

template <typename Real>
void launch_adam(int64_t P, Real* theta, Real* m, Real* v, const Real* g, double lr, double beta1,
                 double beta2, double eps, const long long* t_dev, hipStream_t st) {
  k_adam<Real><<<cdiv(P, 256), 256, 0, st>>>(P, theta, m, v, g, lr, beta1, beta2, eps, t_dev);
}

#define CRV_INST(R)                                                                            \
  template void launch_mlp_forward<R>(const Geom&, const MlpShape&, const R*, R*, long long*,    \
                                      hipStream_t);                                            \
  template int launch_mlp_backward<R>(const Geom&, const MlpShape&, const R*, const R*, R*,    \
                                      hipStream_t);                                            \
  template void launch_reduce_rows<R>(const R*, int, int64_t, int64_t, R*, R*, hipStream_t);            \
  template void launch_adam<R>(int64_t, R*, R*, R*, const R*, double, double, double, double,  \
                               const long long*, hipStream_t);
CRV_INST(float)
CRV_INST(double)

}  // namespace crv
