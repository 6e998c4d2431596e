// Matrix-core (MFMA) formulation of the pressure network u = m NN_theta(2x-1)
// for float32 (v_mfma_f32_32x32x2f32) and bf16 (v_mfma_f32_32x32x16_bf16,
// float32 accumulate).
//
// Layout.  Activations are kept transposed, features x nodes, in 32 x 32
// accumulator tiles: a wavefront owns 32 nodes (one per lane column) and lane
// group g = lane/32 holds, for every 32-feature block mb, the 16 features
// 32 mb + 8 (i/4) + 4 g + (i%4), i = 0..15 (the accumulator layout of the
// 32x32 MFMA).  A layer's output registers are directly the B operand of the
// next layer's product: K-step ks takes the lane's registers
// ks*S .. ks*S+S-1 (S = 8 for bf16, 1 for fp32), so the contraction index
// runs over features in a lane-dependent order.  That order is folded into
// the packed weight fragments (k_pack_fragments), so no data moves between
// layers.  Bias is added by initialising the accumulators with it; tanh is
// applied in float32 on the vector ALUs.
//
// Backward.  delta_{l-1} = (W_l^T delta_l) (1 - h_{l-1}^2) uses the same
// register chain with transposed fragments.  The weight gradient
// dW_l = sum_nodes delta_l h_{l-1}^T contracts over nodes: the waves of a
// block write delta_l and h_{l-1} of their tiles transposed into LDS, and each
// wave accumulates its share of the dW_l output tiles with MFMAs over the
// block's nodes.  Accumulators persist in registers across the block's
// node tiles; each block writes one partial gradient row at the end, reduced
// in a fixed order afterwards.  Small gradients (biases, first and last
// layer) are summed per thread from LDS.
#include <algorithm>

#include "kernels.h"

namespace crv {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

template <bool BF16>
struct MM;

template <>
struct MM<true> {
  static constexpr int S = 8;    // operand values per lane
  static constexpr int KS = 16;  // contraction length per instruction
  using elem = __bf16;
  using op = bf16x8_t;
  __device__ static inline f32x16_t mma(op a, op b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static inline op load(const elem* p) { return *reinterpret_cast<const op*>(p); }
  __device__ static inline op from(const float* v) {
    op o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = (__bf16)v[k];
    return o;
  }
};

template <>
struct MM<false> {
  static constexpr int S = 1;
  static constexpr int KS = 2;
  using elem = float;
  using op = float;
  __device__ static inline f32x16_t mma(op a, op b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline op load(const elem* p) { return *p; }
  __device__ static inline op from(const float* v) { return v[0]; }
};

// feature held by lane group g in its flat accumulator register t (t = 16 mb + i)
__host__ __device__ inline int cfeat(int t, int g) {
  return 32 * (t >> 4) + 8 * ((t & 15) >> 2) + 4 * g + (t & 3);
}

__host__ __device__ inline int64_t off_layer(int l, int dim, int W) {
  // parameter offset of hidden layer l (1-based); l = hidden+1 is the output layer
  return l == 1 ? 0 : int64_t(W) * dim + W + int64_t(l - 2) * (int64_t(W) * W + W);
}

// ---------------------------------------------------------------------------
// Packed fragments: for hidden-to-hidden layer hl (layer l = hl + 2), block mb
// and K-step ks, lane (r = lane%32, g = lane/32) holds S consecutive values:
//   forward  (dir 0): W_l[32 mb + r][cfeat(ks*S + v, g)]
//   backward (dir 1): W_l[cfeat(ks*S + v, g)][32 mb + r]      (= W_l^T)
// index (((hl*2 + dir) * (W/32) + mb) * (W/KS) + ks) * 64*S + lane*S + v.
// ---------------------------------------------------------------------------
template <bool BF16>
__global__ void k_pack_fragments(const float* __restrict__ th, int dim, int W, int hidden,
                                 typename MM<BF16>::elem* __restrict__ frag) {
  using T = MM<BF16>;
  const int64_t per_layer = 2 * int64_t(W) * W;
  const int64_t total = per_layer * (hidden - 1);
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int v = int(idx % T::S);
  const int lane = int((idx / T::S) % 64);
  int64_t rest = idx / (T::S * 64);
  const int nks = W / T::KS;
  const int ks = int(rest % nks);
  rest /= nks;
  const int mb = int(rest % (W / 32));
  rest /= (W / 32);
  const int dir = int(rest % 2);
  const int hl = int(rest / 2);
  const int r = lane & 31, g = lane >> 5;
  const int a = 32 * mb + r;                 // row of the A operand
  const int k = cfeat(ks * T::S + v, g);     // contraction feature
  const float* Wl = th + off_layer(hl + 2, dim, W);
  const float w = dir == 0 ? Wl[int64_t(a) * W + k] : Wl[int64_t(k) * W + a];
  frag[idx] = typename MM<BF16>::elem(w);
}

template <int DIM>
__device__ inline void node_z(int64_t p, int n, int ne, float* z, bool* interior) {
  const int i = int(p % n), j = int((p / n) % n);
  const double inv = 1.0 / double(ne);
  z[0] = float(2.0 * (double(i) * inv) - 1.0);
  z[1] = float(2.0 * (double(j) * inv) - 1.0);
  bool in = i > 0 && i < ne && j > 0 && j < ne;
  if (DIM == 3) {
    const int k = int(p / (int64_t(n) * n));
    z[DIM - 1] = float(2.0 * (double(k) * inv) - 1.0);
    in = in && k > 0 && k < ne;
  }
  *interior = in;
}

// Small parameters staged in LDS per block: W1 (W x DIM), b1, the hidden
// biases b_2..b_L, w_out, b_out -- W (DIM + L + 1) + 1 floats.
template <int W, int L, int DIM>
struct Small {
  static constexpr int W1 = 0, B1 = W * DIM, BH = B1 + W, WO = BH + (L - 1) * W, BO = WO + W;
  static constexpr int SIZE = BO + 1;
  __device__ static void stage(const float* th, float* sp, int tid, int nth) {
    for (int k = tid; k < SIZE; k += nth) {
      float v;
      if (k < B1 + W) v = th[k];                                   // W1, b1 (contiguous)
      else if (k < WO) {
        const int l = (k - BH) / W + 2, f = (k - BH) % W;          // bias of hidden layer l
        v = th[off_layer(l, DIM, W) + int64_t(W) * W + f];
      } else v = th[off_layer(L + 1, DIM, W) + (k - WO)];          // w_out, b_out
      sp[k] = v;
    }
  }
};

// Forward of one 32-node tile held by this wave.  Every hidden layer's
// activations (accumulator layout, float32) are handed to sink(l, h) as soon
// as they are computed; on return h holds the last hidden layer.
struct NoSink {
  template <typename H>
  __device__ void operator()(int, const H&) const {}
};

template <int W, int L, bool BF16, int DIM, typename Sink>
__device__ inline void forward_tile(const float* sp,
                                    const typename MM<BF16>::elem* __restrict__ frag,
                                    const float* z, int g, int lane, float (&h)[W / 2],
                                    const Sink& sink) {
  using T = MM<BF16>;
  using SM = Small<W, L, DIM>;
  constexpr int NR = W / 2;          // accumulator registers per lane
  constexpr int NKS = W / T::KS;     // K-steps per layer
  constexpr int NMB = W / 32;
  // layer 1 on the vector ALUs (K = DIM)
  {
    const float* W1 = sp + SM::W1;
    const float* b1 = sp + SM::B1;
#pragma unroll
    for (int t = 0; t < NR; ++t) {
      const int f = cfeat(t, g);
      float a = b1[f];
#pragma unroll
      for (int c = 0; c < DIM; ++c) a += W1[f * DIM + c] * z[c];
      h[t] = tanh_fast(a);
    }
    sink(0, h);
  }
#pragma unroll
  for (int l = 1; l < L; ++l) {
    const float* bl = sp + SM::BH + (l - 1) * W;
    typename T::op bop[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) bop[ks] = T::from(&h[ks * T::S]);
    f32x16_t acc[NMB];
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[mb][i] = bl[cfeat(mb * 16 + i, g)];
    const typename T::elem* fl = frag + int64_t((l - 1) * 2 + 0) * NMB * NKS * 64 * T::S;
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks)
        acc[mb] = T::mma(T::load(fl + (int64_t(mb) * NKS + ks) * 64 * T::S + lane * T::S), bop[ks],
                         acc[mb]);
#pragma unroll
    for (int t = 0; t < NR; ++t) h[t] = tanh_fast(acc[t >> 4][t & 15]);
    sink(l, h);
  }
}

template <int W, int L, bool BF16, int DIM>
__global__ __launch_bounds__(256) void k_mlp_fwd_mfma(Geom geo, const float* __restrict__ th,
                                                      const typename MM<BF16>::elem* __restrict__ frag,
                                                      float* __restrict__ u, long long* t_bump) {
  constexpr int NR = W / 2;
  using SM = Small<W, L, DIM>;
  if (t_bump && blockIdx.x == 0 && threadIdx.x == 0) *t_bump = *t_bump + 1;  // new Adam iteration
  __shared__ float sp[SM::SIZE];
  SM::stage(th, sp, threadIdx.x, blockDim.x);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 5, n = lane & 31;
  const int64_t total = ipow(geo.n, DIM);
  const int64_t tile = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int64_t p = tile * 32 + n;
  if (tile * 32 >= total) return;  // whole wave leaves together
  float z[DIM];
  bool interior = false;
  if (p < total) node_z<DIM>(p, geo.n, geo.ne, z, &interior);
  else
    for (int c = 0; c < DIM; ++c) z[c] = 0.f;
  float h[NR];
  forward_tile<W, L, BF16, DIM>(sp, frag, z, g, lane, h, NoSink());
  const float* wo = sp + SM::WO;
  float s = 0.f;
#pragma unroll
  for (int t = 0; t < NR; ++t) s += wo[cfeat(t, g)] * h[t];
  s += __shfl_xor(s, 32, 64);
  if (g == 0 && p < total) u[p] = interior ? s + wo[W] : 0.f;
}

// ---------------------------------------------------------------------------
// Backward.  Block = NW waves, a block step covers NB = 32*NW nodes.  The
// recomputed activations of every hidden layer go to LDS transposed
// (Hall[l][feature][node]); that copy is the B operand of the dW products
// and the source of the tanh derivative, so only one layer is live in
// registers at a time.
// ---------------------------------------------------------------------------
template <int W, int L, bool BF16, int DIM, int NW>
__global__ __launch_bounds__(64 * NW) void k_mlp_bwd_mfma(Geom geo, int64_t P,
                                                          const float* __restrict__ th,
                                                          const typename MM<BF16>::elem* __restrict__ frag,
                                                          const float* __restrict__ gu,
                                                          float* __restrict__ partials) {
  using T = MM<BF16>;
  using E = typename T::elem;
  constexpr int NR = W / 2, NKS = W / T::KS, NMB = W / 32;
  constexpr int NB = 32 * NW;                 // nodes per block step
  constexpr int PAD = BF16 ? 8 : 1;
  constexpr int LD = NB + PAD;                // row pitch of the transposed buffers
  constexpr int NOB = NMB * NMB;              // 32x32 output tiles of one dW_l
  constexpr int OWN = (NOB + NW - 1) / NW;    // tiles owned by each wave
  constexpr int NTH = 64 * NW;
  constexpr int FPT = (W * 4 + NTH - 1) / NTH;  // features per thread (4 quarters per feature)
  constexpr int QN = NB / 4;                  // nodes per quarter
  __shared__ __attribute__((aligned(16))) E Hall[L * W * LD];
  __shared__ __attribute__((aligned(16))) E Dt[W * LD];
  __shared__ float Gs[NB];
  __shared__ float Zs[DIM][NB];
  __shared__ float Red[NTH];
  using SM = Small<W, L, DIM>;
  __shared__ float sp[SM::SIZE];

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 5, n = lane & 31;
  const int col = w * 32 + n;  // this lane's node column in the block step
  SM::stage(th, sp, tid, NTH);
  __syncthreads();
  const int64_t total = ipow(geo.n, DIM);
  const int64_t nsteps = (total + NB - 1) / NB;

  f32x16_t acc[L - 1][OWN];
#pragma unroll
  for (int a = 0; a < L - 1; ++a)
#pragma unroll
    for (int o = 0; o < OWN; ++o)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][o][i] = 0.f;
  // per-thread small gradients: feature fq = tid/4 + f*(NTH/4), node quarter tid%4
  float s_wout[FPT], s_b[L][FPT], s_w1[DIM][FPT], s_bout = 0.f;
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    s_wout[f] = 0.f;
#pragma unroll
    for (int l = 0; l < L; ++l) s_b[l][f] = 0.f;
#pragma unroll
    for (int c = 0; c < DIM; ++c) s_w1[c][f] = 0.f;
  }
  const int q = tid & 3;
  const float* wo = sp + SM::WO;
  auto sink = [&](int l, const float(&hv)[NR]) {
#pragma unroll
    for (int t = 0; t < NR; ++t) Hall[(l * W + cfeat(t, g)) * LD + col] = E(hv[t]);
  };

  for (int64_t step = blockIdx.x; step < nsteps; step += gridDim.x) {
    const int64_t p = step * NB + col;
    float z[DIM];
    bool interior = false;
    const bool valid = p < total;
    if (valid) node_z<DIM>(p, geo.n, geo.ne, z, &interior);
    else
      for (int c = 0; c < DIM; ++c) z[c] = 0.f;
    float d[NR];
    forward_tile<W, L, BF16, DIM>(sp, frag, z, g, lane, d, sink);
    const float gv = valid ? gu[p] : 0.f;
    if (g == 0) {
      Gs[col] = gv;
#pragma unroll
      for (int c = 0; c < DIM; ++c) Zs[c][col] = z[c];
    }
    // delta of the last hidden layer: g w_out (1 - h_L^2), h_L still in d
#pragma unroll
    for (int t = 0; t < NR; ++t) d[t] = gv * wo[cfeat(t, g)] * (1.f - d[t] * d[t]);
    __syncthreads();
    // output layer: dW_out[f] = sum_n g_n h_L[f][n], db_out = sum_n g_n
#pragma unroll
    for (int f = 0; f < FPT; ++f) {
      const int fq = (tid >> 2) + f * (NTH / 4);
      if (fq < W) {
        const E* hr = Hall + ((L - 1) * W + fq) * LD + q * QN;
        float s = 0.f;
        for (int k = 0; k < QN; ++k) s += float(hr[k]) * Gs[q * QN + k];
        s_wout[f] += s;
      }
    }
    if (tid < 4) {
      float s = 0.f;
      for (int k = 0; k < QN; ++k) s += Gs[tid * QN + k];
      s_bout += s;
    }
#pragma unroll
    for (int l = L; l >= 1; --l) {
      // delta_l transposed into LDS
#pragma unroll
      for (int t = 0; t < NR; ++t) Dt[cfeat(t, g) * LD + col] = E(d[t]);
      __syncthreads();
      if (l >= 2) {
        // dW_l[o][i] += sum_nodes delta_l[o][node] h_{l-1}[i][node]
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
          const int tileid = w * OWN + o;
          if (tileid < NOB) {
            const int ob = tileid / NMB, ib = tileid % NMB;
            const E* arow = Dt + (ob * 32 + n) * LD + T::S * g;
            const E* brow = Hall + ((l - 2) * W + ib * 32 + n) * LD + T::S * g;
#pragma unroll
            for (int ks = 0; ks < NB / T::KS; ++ks)
              acc[l - 2][o] = T::mma(T::load(arow + ks * T::KS), T::load(brow + ks * T::KS),
                                     acc[l - 2][o]);
          }
        }
      }
#pragma unroll
      for (int f = 0; f < FPT; ++f) {
        const int fq = (tid >> 2) + f * (NTH / 4);
        if (fq < W) {
          const E* dr = Dt + fq * LD + q * QN;
          float sb = 0.f;
          float sw[DIM];
#pragma unroll
          for (int c = 0; c < DIM; ++c) sw[c] = 0.f;
          for (int k = 0; k < QN; ++k) {
            const float dv = float(dr[k]);
            sb += dv;
            if (l == 1)
#pragma unroll
              for (int c = 0; c < DIM; ++c) sw[c] += dv * Zs[c][q * QN + k];
          }
          s_b[l - 1][f] += sb;
          if (l == 1)
#pragma unroll
            for (int c = 0; c < DIM; ++c) s_w1[c][f] += sw[c];
        }
      }
      if (l >= 2) {
        // delta_{l-1} = (W_l^T delta_l) (1 - h_{l-1}^2)
        typename T::op bop[NKS];
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) bop[ks] = T::from(&d[ks * T::S]);
        const E* fl = frag + int64_t((l - 2) * 2 + 1) * NMB * NKS * 64 * T::S;
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
          f32x16_t c2;
#pragma unroll
          for (int i = 0; i < 16; ++i) c2[i] = 0.f;
#pragma unroll
          for (int ks = 0; ks < NKS; ++ks)
            c2 = T::mma(T::load(fl + (int64_t(mb) * NKS + ks) * 64 * T::S + lane * T::S), bop[ks], c2);
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const float hv = float(Hall[((l - 2) * W + cfeat(mb * 16 + i, g)) * LD + col]);
            d[mb * 16 + i] = c2[i] * (1.f - hv * hv);
          }
        }
      }
      __syncthreads();
    }
  }

  // ---- write this block's partial gradient row ----
  float* row = partials + int64_t(blockIdx.x) * P;
#pragma unroll
  for (int l = 2; l <= L; ++l) {
    const int64_t off = off_layer(l, DIM, W);
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
      const int tileid = w * OWN + o;
      if (tileid < NOB) {
        const int ob = tileid / NMB, ib = tileid % NMB;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int orow = ob * 32 + 8 * (i >> 2) + 4 * g + (i & 3);
          const int icol = ib * 32 + n;
          row[off + int64_t(orow) * W + icol] = acc[l - 2][o][i];
        }
      }
    }
  }
  // small gradients: reduce the four quarters of each feature through LDS
  auto reduce4 = [&](float v, int64_t dst, bool ok) {
    Red[tid] = v;
    __syncthreads();
    if (ok && q == 0) row[dst] = Red[tid] + Red[tid + 1] + Red[tid + 2] + Red[tid + 3];
    __syncthreads();
  };
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    const int fq = (tid >> 2) + f * (NTH / 4);
    const bool ok = fq < W;
    reduce4(s_wout[f], off_layer(L + 1, DIM, W) + fq, ok);
#pragma unroll
    for (int l = 1; l <= L; ++l) {
      const int in_dim = l == 1 ? DIM : W;
      reduce4(s_b[l - 1][f], off_layer(l, DIM, W) + int64_t(W) * in_dim + fq, ok);
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) reduce4(s_w1[c][f], int64_t(fq) * DIM + c, ok);
  }
  // threads 0..3 each summed one quarter of g: combine them for the output bias
  Red[tid] = (tid < 4) ? s_bout : 0.f;
  __syncthreads();
  if (tid == 0) row[off_layer(L + 1, DIM, W) + W] = Red[0] + Red[1] + Red[2] + Red[3];
}

// ---------------------------------------------------------------------------
// Fused gradient reduction + Adam + fragment update.  Block = 4 waves over
// 64 parameters (one per lane); wave w sums partial rows w, w+4, ... and the
// four wave sums are added in a fixed order.  The updated weight of a
// hidden-to-hidden layer is written straight into its two fragment slots
// (the inverse of the k_pack_fragments map).
// ---------------------------------------------------------------------------
// flat accumulator register t and lane group g holding feature f (cfeat inverse)
__device__ inline void cfeat_inv(int f, int* t, int* g) {
  *g = (f >> 2) & 1;
  *t = 16 * (f >> 5) + 4 * ((f & 31) >> 3) + (f & 3);
}

template <bool BF16>
__global__ __launch_bounds__(256) void k_reduce_adam_pack(
    const float* __restrict__ part, int rows, int64_t P, float* __restrict__ th,
    float* __restrict__ m, float* __restrict__ v, double lr, double b1, double b2, double eps,
    const long long* __restrict__ t_dev, int dim, int W, int hidden,
    typename MM<BF16>::elem* __restrict__ frag, const float* __restrict__ loss_part, int loss_np,
    double* __restrict__ hist, int cap) {
  using T = MM<BF16>;
  __shared__ float red[4][64];
  if (blockIdx.x == gridDim.x - 1) {
    // the extra block: loss of this iteration (fixed-order sum of the partials)
    __shared__ double lb[256];
    double v = 0;
    for (int k = threadIdx.x; k < loss_np; k += 256) v += double(loss_part[k]);
    const double tot = block_sum(v, lb);
    if (threadIdx.x == 0) hist[(*t_dev - 1) % cap] = tot;
    return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t p = int64_t(blockIdx.x) * 64 + lane;
  float s = 0.f;
  if (p < P) {
    int r = w;
    for (; r + 12 < rows; r += 16) {
      const float a0 = part[int64_t(r) * P + p], a1 = part[int64_t(r + 4) * P + p];
      const float a2 = part[int64_t(r + 8) * P + p], a3 = part[int64_t(r + 12) * P + p];
      s += a0;
      s += a1;
      s += a2;
      s += a3;
    }
    for (; r < rows; r += 4) s += part[int64_t(r) * P + p];
  }
  red[w][lane] = s;
  __syncthreads();
  if (w != 0 || p >= P) return;
  const float gg = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
  const double t = double(*t_dev);
  const float c1 = float(1.0 - pow(b1, t)), c2 = float(1.0 - pow(b2, t));
  const float mm = float(b1) * m[p] + float(1.0 - b1) * gg;
  const float vv = float(b2) * v[p] + float(1.0 - b2) * gg * gg;
  m[p] = mm;
  v[p] = vv;
  const float nw = th[p] - float(lr) * (mm / c1) / (sqrtf(vv / c2) + float(eps));
  th[p] = nw;
  if (frag == nullptr) return;
  // hidden-to-hidden weight? layer l = 2..hidden occupies [off_l, off_l + W*W)
  const int64_t base = int64_t(W) * dim + W;
  if (p < base) return;
  const int64_t rel = p - base, per = int64_t(W) * W + W;
  const int hl = int(rel / per);
  const int64_t within = rel % per;
  if (hl >= hidden - 1 || within >= int64_t(W) * W) return;
  const int o = int(within / W), i = int(within % W);
  const int nks = W / T::KS, nmb = W / 32;
  const typename MM<BF16>::elem e = typename MM<BF16>::elem(nw);
  int tt, g;
  // forward fragment: row o, contraction feature i
  cfeat_inv(i, &tt, &g);
  {
    const int ks = tt / T::S, vv2 = tt % T::S, mb = o >> 5, lanei = (o & 31) + 32 * g;
    frag[((((int64_t(hl) * 2 + 0) * nmb + mb) * nks + ks) * 64 + lanei) * T::S + vv2] = e;
  }
  // backward (transposed) fragment: row i, contraction feature o
  cfeat_inv(o, &tt, &g);
  {
    const int ks = tt / T::S, vv2 = tt % T::S, mb = i >> 5, lanei = (i & 31) + 32 * g;
    frag[((((int64_t(hl) * 2 + 1) * nmb + mb) * nks + ks) * 64 + lanei) * T::S + vv2] = e;
  }
}

void launch_reduce_adam_pack(const float* partials, int rows, int64_t P, float* theta, float* m,
                             float* v, double lr, double b1, double b2, double eps,
                             const long long* t_dev, int dim, int width, int hidden, bool bf16,
                             void* frag, const float* loss_part, int loss_np, double* loss_hist,
                             int cap, hipStream_t st) {
  const int blocks = cdiv(P, 64) + 1;
  if (bf16)
    k_reduce_adam_pack<true><<<blocks, 256, 0, st>>>(partials, rows, P, theta, m, v, lr, b1, b2, eps,
                                                     t_dev, dim, width, hidden,
                                                     static_cast<__bf16*>(frag), loss_part, loss_np,
                                                     loss_hist, cap);
  else
    k_reduce_adam_pack<false><<<blocks, 256, 0, st>>>(partials, rows, P, theta, m, v, lr, b1, b2, eps,
                                                      t_dev, dim, width, hidden,
                                                      static_cast<float*>(frag), loss_part, loss_np,
                                                      loss_hist, cap);
}

// ---------------------------------------------------------------------------
bool mlp_mfma_supported(int dim, int width, int hidden, bool bf16) {
  if (dim != 2) return false;
  if (!(hidden == 3 || hidden == 4)) return false;
  (void)bf16;
  return width == 32 || width == 64;
}

int64_t mlp_fragment_elems(int width, int hidden) { return 2 * int64_t(width) * width * (hidden - 1); }

void launch_pack_fragments(const float* theta, int dim, int width, int hidden, bool bf16,
                           void* frag, hipStream_t st) {
  const int64_t total = mlp_fragment_elems(width, hidden);
  if (total <= 0) return;
  if (bf16)
    k_pack_fragments<true><<<cdiv(total, 256), 256, 0, st>>>(theta, dim, width, hidden,
                                                             static_cast<__bf16*>(frag));
  else
    k_pack_fragments<false><<<cdiv(total, 256), 256, 0, st>>>(theta, dim, width, hidden,
                                                              static_cast<float*>(frag));
}

template <int W, int L, bool BF16>
static void fwd_inst(const Geom& g, const float* th, const void* frag, float* u, long long* tb,
                     hipStream_t st) {
  const int64_t total = ipow(g.n, 2);
  const int64_t tiles = (total + 31) / 32;
  k_mlp_fwd_mfma<W, L, BF16, 2><<<cdiv(tiles, 4), 256, 0, st>>>(
      g, th, static_cast<const typename MM<BF16>::elem*>(frag), u, tb);
}

void launch_mlp_forward_mfma(const Geom& g, int width, int hidden, bool bf16, const float* theta,
                             const void* frag, float* u, long long* t_bump, hipStream_t st) {
#define CRV_FW(WW, LL, BB) \
  if (width == WW && hidden == LL && bf16 == BB) return fwd_inst<WW, LL, BB>(g, theta, frag, u, t_bump, st);
  CRV_FW(32, 3, true) CRV_FW(64, 3, true)
  CRV_FW(32, 4, true) CRV_FW(64, 4, true)
  CRV_FW(32, 3, false) CRV_FW(64, 3, false) CRV_FW(32, 4, false) CRV_FW(64, 4, false)
#undef CRV_FW
}

// waves per backward block: bf16 activations fit 4 waves' worth of nodes in
// LDS, float32 ones 2
constexpr int bwd_nw(bool bf16) { return bf16 ? 4 : 2; }

int mlp_bwd_mfma_blocks(const Geom& g, bool bf16, int cu_count) {
  const int64_t total = ipow(g.n, g.dim);
  const int nb = 32 * bwd_nw(bf16);
  const int64_t steps = (total + nb - 1) / nb;
  return int(std::max<int64_t>(1, std::min<int64_t>(steps, cu_count)));
}

template <int W, int L, bool BF16>
static void bwd_inst(const Geom& g, int64_t P, const float* th, const void* frag, const float* gu,
                     float* partials, int blocks, hipStream_t st) {
  constexpr int NW = bwd_nw(BF16);
  k_mlp_bwd_mfma<W, L, BF16, 2, NW><<<blocks, 64 * NW, 0, st>>>(
      g, P, th, static_cast<const typename MM<BF16>::elem*>(frag), gu, partials);
}

void launch_mlp_backward_mfma(const Geom& g, int width, int hidden, bool bf16, int64_t P,
                              const float* theta, const void* frag, const float* gu,
                              float* partials, int blocks, hipStream_t st) {
#define CRV_BW(WW, LL, BB) \
  if (width == WW && hidden == LL && bf16 == BB) return bwd_inst<WW, LL, BB>(g, P, theta, frag, gu, partials, blocks, st);
  CRV_BW(32, 3, true) CRV_BW(64, 3, true)
  CRV_BW(32, 4, true) CRV_BW(64, 4, true)
  CRV_BW(32, 3, false) CRV_BW(64, 3, false) CRV_BW(32, 4, false) CRV_BW(64, 4, false)
#undef CRV_BW
}

}  // namespace crv
