// Matrix-core (MFMA) formulation of the pressure network u = m NN_theta(2x-1).
//
// Three arithmetic modes for the hidden-to-hidden products (float32
// accumulation in all of them):
//   F32   v_mfma_f32_16x16x4f32 on float32 operands;
//   BF16  v_mfma_f32_16x16x32_bf16 on bf16-rounded operands;
//   X3    split bf16: every operand a = a_hi + a_lo with a_hi = bf16(a),
//         a_lo = bf16(a - a_hi), and a.b ~ a_hi.b_hi + a_hi.b_lo + a_lo.b_hi
//         (three bf16 MFMAs, about 2^-16 relative error per product).
// The first layer (K = d) and the output (N = 1) run on the vector ALUs in
// float32, as do tanh and its derivative.
//
// Layout.  Activations are kept transposed, features x nodes, in 16 x 16
// accumulator tiles: a wavefront owns 16 nodes (lane column r = lane%16) and
// lane group q = lane/16 holds, for every 16-feature block mb, the four
// features 16 mb + 4 q + i, i = 0..3 (the accumulator layout of the 16x16
// MFMA).  A layer's output registers are directly the B operand of the next
// layer's product: K-step ks takes the lane's registers ks*S .. ks*S+S-1
// (S = 8 for bf16, 1 for fp32), so the contraction index runs over features
// in a lane-dependent order.  That order is folded into the packed weight
// fragments, so no data moves between layers.  Bias is added by initialising
// the accumulators with it.  Sixteen nodes per wave keep the per-lane state
// (activations, deltas, weight-gradient tiles) small enough for two or more
// waves per SIMD, so one wave's tanh work overlaps another's matrix products.
//
// Backward.  delta_{l-1} = (W_l^T delta_l) (1 - h_{l-1}^2) uses the same
// register chain with transposed fragments.  dW_l = sum_nodes delta_l
// h_{l-1}^T contracts over nodes: the waves of a block write delta_l
// transposed into LDS next to the recomputed activations (also transposed),
// and each wave accumulates its share of the 16x16 dW_l output tiles with
// MFMAs over the block's nodes.  Biases, first-layer and output weights are
// summed over nodes per thread from LDS.  All accumulators persist across the
// block's node tiles; each block writes one partial gradient row, reduced in
// a fixed order afterwards.
#include <algorithm>

#include "kernels.h"
#include "stencil.h"

namespace crv {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// Two floats rounded to bf16 (nearest even) by one conversion into one
// register, v0 in the low half and v1 in the high half.  The empty asm makes
// the pair opaque, so every later use of a half (its float value, a 16-bit
// store) is taken from this register by a shift, a mask or a high-half store,
// instead of the compiler converting that float a second time on its own.
__device__ inline unsigned int bf16_pair(float v0, float v1) {
  unsigned int w = __builtin_bit_cast(unsigned int, __builtin_convertvector(f32x2_t{v0, v1}, bf16x2_t));
  asm("" : "+v"(w));
  return w;
}
// the float values of the two halves (exact)
__device__ inline float bf16_lo_float(unsigned int w) { return __builtin_bit_cast(float, w << 16); }
__device__ inline float bf16_hi_float(unsigned int w) { return __builtin_bit_cast(float, w & 0xffff0000u); }
__device__ inline void put_bits(__bf16* p, unsigned int bits16) {
  *reinterpret_cast<unsigned short*>(p) = (unsigned short)bits16;
}
// bf16 element v of a packed eight-value operand
__device__ inline void put_elem(__bf16* p, const bf16x8_t& o, int v) {
  const unsigned int w = __builtin_bit_cast(u32x4_t, o)[v >> 1];
  put_bits(p, (v & 1) ? (w >> 16) : w);
}
// eight floats rounded to bf16 as one operand (four paired conversions)
__device__ inline bf16x8_t bf16x8_from(const float* v) {
  u32x4_t w;
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = bf16_pair(v[2 * k], v[2 * k + 1]);
  return __builtin_bit_cast(bf16x8_t, w);
}

template <int M>
struct MM;

template <>
struct MM<NET_F32> {
  static constexpr int S = 1, KS = 4, NP = 1;  // values per lane, K per MFMA, fragment planes
  using felem = float;                          // fragment storage
  using lelem = float;                          // LDS storage of activations / deltas
  static constexpr int PAD = 4;
  using op = float;
  __device__ static inline f32x4_t mma(op a, op b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  using wop = op;  // weight operand
  __device__ static inline f32x4_t mma_w(wop a, op b, f32x4_t c) { return mma(a, b, c); }
  static constexpr int NPL = 1;                 // LDS planes per value
  __device__ static inline op frag(const felem* p) { return *p; }
  __device__ static inline op from(const float* v) { return v[0]; }
  __device__ static inline void put(felem* p, float w) { p[0] = w; }
  __device__ static inline f32x4_t row_sum(op a, f32x4_t c) { return mma(a, 1.0f, c); }
  __device__ static inline op lds_op(const lelem* p, int) { return *p; }
  __device__ static inline float lds_get(const lelem* p, int) { return *p; }
  __device__ static inline void lds_put(lelem* p, int, float v) { *p = v; }
  __device__ static inline void lds_put2(lelem* p0, lelem* p1, int, float v0, float v1) {
    *p0 = v0;
    *p1 = v1;
  }
  __device__ static inline void lds_put_elem(lelem* p, int, const op& o, int) { *p = o; }
};

template <>
struct MM<NET_BF16> {
  static constexpr int S = 8, KS = 32, NP = 1;
  using felem = __bf16;
  using lelem = __bf16;
  static constexpr int PAD = 8;
  using op = bf16x8_t;
  __device__ static inline f32x4_t mma(op a, op b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  using wop = op;
  __device__ static inline f32x4_t mma_w(wop a, op b, f32x4_t c) { return mma(a, b, c); }
  static constexpr int NPL = 1;
  __device__ static inline op frag(const felem* p) { return *reinterpret_cast<const op*>(p); }
  __device__ static inline op from(const float* v) { return bf16x8_from(v); }
  __device__ static inline void put(felem* p, float w) { p[0] = (__bf16)w; }
  __device__ static inline f32x4_t row_sum(op a, f32x4_t c) {
    op one;
#pragma unroll
    for (int k = 0; k < 8; ++k) one[k] = (__bf16)1.0f;
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, one, c, 0, 0, 0);
  }
  __device__ static inline op lds_op(const lelem* p, int) { return *reinterpret_cast<const op*>(p); }
  __device__ static inline float lds_get(const lelem* p, int) { return float(*p); }
  __device__ static inline void lds_put(lelem* p, int, float v) { *p = (__bf16)v; }
  __device__ static inline void lds_put2(lelem* p0, lelem* p1, int, float v0, float v1) {
    const unsigned int w = bf16_pair(v0, v1);
    put_bits(p0, w);
    put_bits(p1, w >> 16);
  }
  __device__ static inline void lds_put_elem(lelem* p, int, const op& o, int v) { put_elem(p, o, v); }
};

struct SplitOp {
  bf16x8_t h, l;
};

// LDS holds X3 activations and deltas already split: a hi plane and, `plane`
// elements further, a lo plane, so the weight-gradient products read ready
// operands and the split is done once per value (by the writer).
template <>
struct MM<NET_X3> {
  static constexpr int S = 8, KS = 32, NP = 2;
  using felem = __bf16;
  using lelem = __bf16;
  static constexpr int PAD = 8;
  static constexpr int NPL = 2;
  using op = SplitOp;
  __device__ static inline f32x4_t mma(const op& a, const op& b, f32x4_t c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
  }
  using wop = op;
  __device__ static inline f32x4_t mma_w(const wop& a, const op& b, f32x4_t c) { return mma(a, b, c); }
  // fragments hold the hi plane, then (64*S further) the lo plane
  __device__ static inline op frag(const felem* p) {
    return op{*reinterpret_cast<const bf16x8_t*>(p), *reinterpret_cast<const bf16x8_t*>(p + 64 * S)};
  }
  __device__ static inline op from(const float* v) {
    u32x4_t wh, wl;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const unsigned int h = bf16_pair(v[2 * k], v[2 * k + 1]);
      wh[k] = h;
      wl[k] = bf16_pair(v[2 * k] - bf16_lo_float(h), v[2 * k + 1] - bf16_hi_float(h));
    }
    return op{__builtin_bit_cast(bf16x8_t, wh), __builtin_bit_cast(bf16x8_t, wl)};
  }
  // the subtraction is kept apart from whatever produced w (no fused
  // multiply-add with a caller's product), so the Adam kernel's in-place
  // fragment update and a repack from theta store the same two halves
  __device__ static inline void put(felem* p, float w) {
#pragma clang fp contract(off)
    const __bf16 h = (__bf16)w;
    p[0] = h;
    p[64 * S] = (__bf16)(w - float(h));
  }
  __device__ static inline f32x4_t row_sum(const op& a, f32x4_t c) {
    bf16x8_t one;
#pragma unroll
    for (int k = 0; k < 8; ++k) one[k] = (__bf16)1.0f;
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, one, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, one, c, 0, 0, 0);
  }
  __device__ static inline op lds_op(const lelem* p, int plane) {
    return op{*reinterpret_cast<const bf16x8_t*>(p), *reinterpret_cast<const bf16x8_t*>(p + plane)};
  }
  __device__ static inline float lds_get(const lelem* p, int plane) {
    return float(p[0]) + float(p[plane]);
  }
  __device__ static inline void lds_put(lelem* p, int plane, float v) {
    const __bf16 h = (__bf16)v;
    p[0] = h;
    p[plane] = (__bf16)(v - float(h));
  }
  __device__ static inline void lds_put2(lelem* p0, lelem* p1, int plane, float v0, float v1) {
    const unsigned int h = bf16_pair(v0, v1);
    const unsigned int l = bf16_pair(v0 - bf16_lo_float(h), v1 - bf16_hi_float(h));
    put_bits(p0, h);
    put_bits(p1, h >> 16);
    put_bits(p0 + plane, l);
    put_bits(p1 + plane, l >> 16);
  }
  __device__ static inline void lds_put_elem(lelem* p, int plane, const op& o, int v) {
    put_elem(p, o.h, v);
    put_elem(p + plane, o.l, v);
  }
};

// Backward of the mixed form: activations and deltas rounded to bf16, weights
// kept split (hi and lo planes of the split-bf16 fragments), so a weight
// product is w_hi.a + w_lo.a (two bf16 MFMAs) and the products of
// activations with deltas (dW, db) are single bf16 MFMAs.  The rounding left is
// that of the activations and deltas (2^-9, not systematic across nodes); the
// weights the backward differentiates are the forward's to 2^-16.
template <>
struct MM<NET_MIX> {
  static constexpr int S = 8, KS = 32, NP = 2;
  using felem = __bf16;
  using lelem = __bf16;
  static constexpr int PAD = 8;
  static constexpr int NPL = 1;
  using op = bf16x8_t;
  __device__ static inline f32x4_t mma(op a, op b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  using wop = SplitOp;
  __device__ static inline f32x4_t mma_w(const wop& w, op b, f32x4_t c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.l, b, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.h, b, c, 0, 0, 0);
  }
  __device__ static inline wop frag(const felem* p) {
    return wop{*reinterpret_cast<const bf16x8_t*>(p), *reinterpret_cast<const bf16x8_t*>(p + 64 * S)};
  }
  __device__ static inline op from(const float* v) { return bf16x8_from(v); }
  __device__ static inline void put(felem* p, float w) { MM<NET_X3>::put(p, w); }
  __device__ static inline f32x4_t row_sum(op a, f32x4_t c) {
    op one;
#pragma unroll
    for (int k = 0; k < 8; ++k) one[k] = (__bf16)1.0f;
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, one, c, 0, 0, 0);
  }

  __device__ static inline op lds_op(const lelem* p, int) { return *reinterpret_cast<const op*>(p); }
  __device__ static inline float lds_get(const lelem* p, int) { return float(*p); }
  __device__ static inline void lds_put(lelem* p, int, float v) { *p = (__bf16)v; }
  __device__ static inline void lds_put2(lelem* p0, lelem* p1, int plane, float v0, float v1) {
    MM<NET_BF16>::lds_put2(p0, p1, plane, v0, v1);
  }
  __device__ static inline void lds_put_elem(lelem* p, int, const op& o, int v) { put_elem(p, o, v); }
};

// tanh(a) = 1 - 2 / (2^(K a) + 1) with K = 2 / ln 2.  Every weight and bias
// that feeds a hidden pre-activation on the forward side (first-layer W1, b1,
// hidden biases, and the forward fragments of the hidden-to-hidden weights)
// is stored pre-multiplied by K, so the products deliver K a directly and the
// activation costs one exp2, one add, one reciprocal and one fma.  The
// transposed (backward) fragments and the output layer are not scaled.
constexpr float kTanhScale = 2.8853900817779268f;

__device__ inline float tanh_of_scaled(float ka) {
  const float e = __builtin_amdgcn_exp2f(ka);
  return __builtin_fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

// feature held by lane group q in its flat accumulator register t (t = 4 mb + i)
__host__ __device__ inline int cfeat(int t, int q) { return 16 * (t >> 2) + 4 * q + (t & 3); }
// inverse: register t and lane group q holding feature f
__host__ __device__ inline void cfeat_inv(int f, int* t, int* q) {
  *q = (f >> 2) & 3;
  *t = 4 * (f >> 4) + (f & 3);
}

__host__ __device__ inline int64_t off_layer(int l, int dim, int W) {
  // parameter offset of hidden layer l (1-based); l = hidden+1 is the output layer
  return l == 1 ? 0 : int64_t(W) * dim + W + int64_t(l - 2) * (int64_t(W) * W + W);
}

// Packed fragments: for hidden-to-hidden layer hl (layer l = hl + 2), block mb
// and K-step ks, lane (r = lane%16, q = lane/16) holds S consecutive values
//   forward  (dir 0): W_l[16 mb + r][cfeat(ks*S + v, q)]
//   backward (dir 1): W_l[cfeat(ks*S + v, q)][16 mb + r]      (= W_l^T)
// at (((hl*2 + dir) * (W/16) + mb) * (W/KS) + ks) * NP*64*S + plane*64*S + lane*S + v.
template <int MODE>
__host__ __device__ inline int64_t frag_index(int hl, int dir, int mb, int ks, int lane, int v, int W) {
  using T = MM<MODE>;
  return (((((int64_t(hl) * 2 + dir) * (W / 16) + mb) * (W / T::KS) + ks) * T::NP) * 64 + lane) * T::S + v;
}

template <int MODE>
__global__ void k_pack_fragments(const float* __restrict__ th, int dim, int W, int hidden,
                                 typename MM<MODE>::felem* __restrict__ frag) {
  using T = MM<MODE>;
  const int64_t total = 2 * int64_t(W) * W * (hidden - 1);
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int v = int(idx % T::S);
  const int lane = int((idx / T::S) % 64);
  int64_t rest = idx / (T::S * 64);
  const int nks = W / T::KS;
  const int ks = int(rest % nks);
  rest /= nks;
  const int mb = int(rest % (W / 16));
  rest /= (W / 16);
  const int dir = int(rest % 2);
  const int hl = int(rest / 2);
  const int r = lane & 15, q = lane >> 4;
  const int a = 16 * mb + r;                 // row of the A operand
  const int k = cfeat(ks * T::S + v, q);     // contraction feature
  const float* Wl = th + off_layer(hl + 2, dim, W);
  const float w = dir == 0 ? kTanhScale * Wl[int64_t(a) * W + k] : Wl[int64_t(k) * W + a];
  T::put(frag + frag_index<MODE>(hl, dir, mb, ks, lane, v, W), w);
}

// network input of node p and its trial-function factor (0 on the boundary)
template <int DIM>
__device__ inline void node_z(int64_t p, int n, int ne, int bfac, float* z, bool* interior,
                              float* fac) {
  int i, j, k;
  node_ijk<DIM>(p, n, &i, &j, &k);
  const double inv = 1.0 / double(ne);
  z[0] = float(2.0 * (double(i) * inv) - 1.0);
  z[1] = float(2.0 * (double(j) * inv) - 1.0);
  bool in = i > 0 && i < ne && j > 0 && j < ne;
  if (DIM == 3) {
    z[DIM - 1] = float(2.0 * (double(k) * inv) - 1.0);
    in = in && k > 0 && k < ne;
  }
  *interior = in;
  *fac = in ? float(trial_factor<DIM>(bfac, ne, i, j, k)) : 0.f;
}

// Small parameters staged in LDS per block: W1 (W x DIM), b1, the hidden
// biases b_2..b_L (these three scaled by kTanhScale), w_out, b_out --
// W (DIM + L + 1) + 1 floats.
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
      sp[k] = k < WO ? kTanhScale * v : v;
    }
  }
};

struct NoSink {
  template <typename H>
  __device__ void operator()(int, const H&) const {}
};

// Layer 1 as a float32 matrix-core product: for row block mb, the 16 x 4
// operand [W1 | b1 | 0] (2D) or [W1 | b1] (3D) times [z; 1; 0] (4 x 16
// nodes) gives the pre-activations in the accumulator layout that the next
// layer reads.  Lane (r = lane%16, q = lane/16) holds A[r][q] and B[q][r].
template <int W, int L, int DIM>
struct Layer1 {
  float a[W / 16];  // this lane's entry of the A operand of each row block
  __device__ void load(const float* sp, int lane) {
    using SM = Small<W, L, DIM>;
    const int r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int mb = 0; mb < W / 16; ++mb) {
      const int f = 16 * mb + r;
      a[mb] = q < DIM ? sp[SM::W1 + f * DIM + q] : (q == DIM ? sp[SM::B1 + f] : 0.f);
    }
  }
};

__device__ inline float layer1_operand(const float* z, int q, int dim) {
  float v = 0.f;
  for (int c = 0; c < 3; ++c)
    if (c < dim && q == c) v = z[c];
  return q == dim ? 1.f : v;
}

// Forward of TPW 16-node tiles held by this wave (the tiles share every
// weight-fragment load and give the wave independent chains of products and
// activations).  The operands that hidden layer l (0-based, l < L-1) feeds
// into the next product go to sink(l, bop) as soon as they are built; on
// return h holds the last hidden layer of every tile.
template <int W, int L, int MODE, int DIM, bool PIPE, int TPW, typename Sink>
__device__ inline void forward_tiles(const float* sp,
                                     const typename MM<MODE>::felem* __restrict__ frag,
                                     const Layer1<W, L, DIM>& l1, const float (&z)[TPW][DIM],
                                     int q, int lane, float (&h)[TPW][W / 4], const Sink& sink) {
  using T = MM<MODE>;
  using SM = Small<W, L, DIM>;
  constexpr int NKS = W / T::KS, NMB = W / 16;
  {
    const f32x4_t zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const float zb = layer1_operand(z[t], q, DIM);
#pragma unroll
      for (int mb = 0; mb < NMB; ++mb) {
        const f32x4_t a = __builtin_amdgcn_mfma_f32_16x16x4f32(l1.a[mb], zb, zero, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) h[t][4 * mb + i] = tanh_of_scaled(a[i]);
      }
    }
  }
#pragma unroll
  for (int l = 1; l < L; ++l) {
    const float* bl = sp + SM::BH + (l - 1) * W;
    typename T::op bop[TPW][NKS];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) bop[t][ks] = T::from(&h[t][ks * T::S]);
    sink(l - 1, bop);
    // one 16-row output block at a time: its activations replace h[.][4mb..4mb+3]
    // (the operands of this layer are already in bop).  With PIPE the
    // products of block mb+1 are issued before the tanh of block mb, so the
    // activation work covers the matrix-core latency (two accumulator tiles
    // live per node tile); without it one, for register-bound callers
    auto products = [&](int mb, f32x4_t (&acc)[TPW]) {
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[t][i] = bl[cfeat(mb * 4 + i, q)];
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const auto f = T::frag(frag + frag_index<MODE>(l - 1, 0, mb, ks, lane, 0, W));
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[t] = T::mma_w(f, bop[t][ks], acc[t]);
      }
    };
    if constexpr (PIPE) {
      f32x4_t cur[TPW], nxt[TPW];
      products(0, cur);
#pragma unroll
      for (int mb = 0; mb < NMB; ++mb) {
        if (mb + 1 < NMB) products(mb + 1, nxt);
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
#pragma unroll
          for (int i = 0; i < 4; ++i) h[t][mb * 4 + i] = tanh_of_scaled(cur[t][i]);
          cur[t] = nxt[t];
        }
      }
    } else {
#pragma unroll
      for (int mb = 0; mb < NMB; ++mb) {
        f32x4_t acc[TPW];
        products(mb, acc);
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) h[t][mb * 4 + i] = tanh_of_scaled(acc[t][i]);
      }
    }
  }
}

// 16-node tiles per wave of the forward: two (shared fragment loads, two
// independent chains) where the registers of two tiles keep four waves per
// SIMD, that is up to width 64
template <int W>
constexpr int fwd_tpw() {
  return W <= 64 ? 2 : 1;
}

template <int W, int L, int MODE, int DIM>
__global__ __launch_bounds__(256) void k_mlp_fwd_mfma(Geom geo, const float* __restrict__ th,
                                                      const typename MM<MODE>::felem* __restrict__ frag,
                                                      float* __restrict__ u, long long* t_bump,
                                                      int64_t zb) {
  th = zofs(th, zb); frag = zofs_flat(frag, zb); u = zofs(u, zb); t_bump = zofs(t_bump, zb);
  constexpr int NR = W / 4;
  using SM = Small<W, L, DIM>;
  if (t_bump && blockIdx.x == 0 && threadIdx.x == 0) *t_bump = *t_bump + 1;  // new Adam iteration
  __shared__ float sp[SM::SIZE];
  SM::stage(th, sp, threadIdx.x, blockDim.x);
  __syncthreads();
  constexpr int TPW = fwd_tpw<W>();
  const int lane = threadIdx.x & 63, q = lane >> 4, n = lane & 15;
  const int64_t total = ipow(geo.n, DIM);
  // tile t of wave w in this block: tile (blockIdx.x * TPW + t) * 4 + w
  const int64_t tile0 = int64_t(blockIdx.x) * 4 * TPW + (threadIdx.x >> 6);
  if (tile0 * 16 >= total) return;  // whole wave leaves together
  float z[TPW][DIM];
  bool interior[TPW];
  float fac[TPW];
  int64_t p[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    p[t] = (tile0 + 4 * t) * 16 + n;
    interior[t] = false;
    fac[t] = 0.f;
    if (p[t] < total) node_z<DIM>(p[t], geo.n, geo.ne, geo.bfac, z[t], &interior[t], &fac[t]);
    else
      for (int c = 0; c < DIM; ++c) z[t][c] = 0.f;
  }
  Layer1<W, L, DIM> l1;
  l1.load(sp, lane);
  float h[TPW][NR];
  forward_tiles<W, L, MODE, DIM, true, TPW>(sp, frag, l1, z, q, lane, h, NoSink());
  const float* wo = sp + SM::WO;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < NR; ++r) s += wo[cfeat(r, q)] * h[t][r];
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    if (q == 0 && p[t] < total) u[p[t]] = interior[t] ? fac[t] * (s + wo[W]) : 0.f;
  }
}

// ---------------------------------------------------------------------------
// Backward.  Block = NW waves of TPW 16-node tiles each, a block step covers
// NB = 16*NW*TPW nodes (tile t of wave w: nodes 16 (t NW + w) .. + 15).  The
// adjoint field g_u = 2 A^T q is evaluated per node from q and alpha (no g_u
// array), and each block also sums its share of LOSS = RES . q into
// loss_part[block].
// Hall[l][feature][node] holds the recomputed activations of hidden layers
// 1..L-1 (the B operands of dW_2..dW_L and the source of the derivative);
// the last layer stays in registers and passes through Dt once for the
// output-weight gradient.  Biases, first-layer and output weights are summed
// over nodes per thread from LDS: thread t owns feature t/4 (+ multiples of
// NTH/4) and a quarter of the block's nodes.
// With two copies of Dt (ND = 2) successive uses of it alternate between
// them, so a use's writes need only the barrier before its reads: the
// readers of the copy being overwritten passed a later barrier first.  The
// node data (g_u, coordinates) alternate by block step for the same reason.
// ---------------------------------------------------------------------------
// waves per SIMD the register allocation must leave room for: plain-bf16
// operands at width <= 64 fit three with one tile per wave, everything else
// two
template <int W, int MODE, int TPW>
constexpr int bwd_min_waves() {
  if (MODE == NET_F32 && W >= 128) return 1;  // float32 weight-gradient tiles: one wave per SIMD
  return ((MODE == NET_BF16 || MODE == NET_MIX) && W <= 64 && TPW == 1) ? 3 : 2;
}

template <int W, int L, int MODE, int DIM, int NW, int TPW>
struct BwdShape {
  using T = MM<MODE>;
  using E = typename T::lelem;
  static constexpr int NB = 16 * NW * TPW;     // nodes per block step
  static constexpr int LD = NB + T::PAD;       // row pitch of the transposed buffers
  static constexpr int NTH = 64 * NW;
  // LDS of one block with nd copies of the delta tile and the node data
  static constexpr size_t bytes(int nd) {
    return sizeof(E) * size_t(T::NPL * ((L - 1) + nd) * W * LD) +
           sizeof(float) * size_t(Small<W, L, DIM>::SIZE + nd * (NB + DIM * NB) + NTH);
  }
  // resident blocks per CU with nd copies: what 160 KB of LDS and the
  // register budget (bwd_min_waves per SIMD) allow (0: does not fit)
  static constexpr int blocks_per_cu(int nd) {
    const int by_lds = int((160u * 1024u) / bytes(nd));
    const int by_regs = bwd_min_waves<W, MODE, TPW>() * 4 / NW;
    const int b = by_lds < by_regs ? by_lds : (by_regs < 1 ? 1 : by_regs);
    return b > 4 ? 4 : b;
  }
  // two copies (one barrier per layer instead of two) whenever they fit and
  // keep the blocks per CU
  static constexpr int ND =
      (blocks_per_cu(2) >= 1 && blocks_per_cu(2) >= blocks_per_cu(1)) ? 2 : 1;
  static constexpr size_t lds_bytes() { return bytes(ND); }
};

template <int W, int L, int MODE, int DIM, int NW, int TPW>
__global__ __launch_bounds__(64 * NW, (bwd_min_waves<W, MODE, TPW>())) void k_mlp_bwd_mfma(Geom geo, int64_t ldp,
                                                             const float* __restrict__ th,
                                                             const typename MM<MODE>::felem* __restrict__ frag,
                                                             const float* __restrict__ qg,
                                                             const float* __restrict__ alpha,
                                                             const float* __restrict__ res,
                                                             float* __restrict__ partials,
                                                             float* __restrict__ loss_part,
                                                             int64_t zb,
                                                             const float* __restrict__ obs_w,
                                                             const float* __restrict__ obs_d,
                                                             const float* __restrict__ u) {
  th = zofs(th, zb); frag = zofs(frag, zb); qg = zofs(qg, zb); alpha = zofs(alpha, zb);
  res = zofs(res, zb); partials = zofs(partials, zb); loss_part = zofs(loss_part, zb);
  obs_w = zofs(obs_w, zb); obs_d = zofs(obs_d, zb); u = zofs(u, zb);
  using T = MM<MODE>;
  using BS = BwdShape<W, L, MODE, DIM, NW, TPW>;
  using E = typename BS::E;
  using SM = Small<W, L, DIM>;
  constexpr int NR = W / 4, NKS = W / T::KS, NMB = W / 16;
  constexpr int NB = BS::NB, LD = BS::LD, NTH = BS::NTH;
  constexpr int NOB = NMB * NMB;              // 16x16 output tiles of one dW_l
  constexpr int OWN = (NOB + NW - 1) / NW;    // tiles owned by each wave
  constexpr int FPT = (W * 4 + NTH - 1) / NTH;  // features per thread
  constexpr int QN = NB / 4;                  // nodes per quarter
  constexpr int HPL = (L - 1) * W * LD, DPL = W * LD;  // plane strides (split storage)
  constexpr int ND = BS::ND;
  __shared__ __attribute__((aligned(16))) E Hall[T::NPL * HPL];
  __shared__ __attribute__((aligned(16))) E Dts[ND][T::NPL * DPL];
  __shared__ float sp[SM::SIZE];
  __shared__ float Gss[ND][NB];
  __shared__ float Zss[ND][DIM][NB];
  __shared__ float Red[NTH];

  // When a wave's tiles do not start a row block at a fixed slot (OWN not a
  // multiple of NMB), which slot holds the bias tile depends on the wave: the
  // wave index is then made a scalar, so that choice is a scalar branch and
  // never an execution mask around a matrix-core instruction (those run on
  // every lane whatever the mask).  Otherwise it is known per slot at compile
  // time and the plain index keeps the register allocation as it is.
  const int tid = threadIdx.x;
  const int w = (OWN % NMB != 0) ? __builtin_amdgcn_readfirstlane(tid >> 6) : (tid >> 6);
  const int lane = tid & 63, q = lane >> 4, n = lane & 15;
  int col[TPW];  // this lane's node column of each of its tiles in the block step
#pragma unroll
  for (int t = 0; t < TPW; ++t) col[t] = (t * NW + w) * 16 + n;
  const int q4 = tid & 3;
  SM::stage(th, sp, tid, NTH);
  __syncthreads();
  Layer1<W, L, DIM> l1;
  l1.load(sp, lane);
  const int64_t total = ipow(geo.n, DIM);
  const int64_t nsteps = (total + NB - 1) / NB;
  const float* wo = sp + SM::WO;
  float lacc = 0.f;  // this lane's share of RES . q (lane group 0 only)

  // a wave's dW tiles cover whole 16-row blocks (OWN a multiple of NMB) or
  // lie inside one; slot o then belongs to row block o / NMB of the wave's
  // (a compile-time index), and each owned row block has its own db tile
  static_assert(OWN % NMB == 0 || NMB % OWN == 0, "dW tiles per wave");
  constexpr int RBW = OWN >= NMB ? OWN / NMB : 1;  // row blocks per wave
  f32x4_t acc[L - 1][OWN];
  f32x4_t bacc[L - 1][RBW];  // db_2..db_L of the wave's row blocks (tile column ib = 0 only)
#pragma unroll
  for (int a = 0; a < L - 1; ++a) {
#pragma unroll
    for (int o = 0; o < OWN; ++o)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[a][o][i] = 0.f;
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) bacc[a][rb][i] = 0.f;
  }
  float s_wout[FPT], s_b[1][FPT], s_w1[DIM][FPT], s_bout = 0.f;
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    s_wout[f] = 0.f;
    s_b[0][f] = 0.f;
#pragma unroll
    for (int c = 0; c < DIM; ++c) s_w1[c][f] = 0.f;
  }
  auto sink = [&](int l, const typename T::op(&bo)[TPW][NKS]) {
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
        for (int v = 0; v < T::S; ++v)
          T::lds_put_elem(Hall + (l * W + cfeat(ks * T::S + v, q)) * LD + col[t], HPL, bo[t][ks], v);
  };

  int ub = 0, gb = 0;  // copy of Dt for the next use; copy of the node data
  for (int64_t step = blockIdx.x; step < nsteps; step += gridDim.x) {
    E* Dt = Dts[ub];
    float* Gs = Gss[gb];
    float(*Zs)[NB] = Zss[gb];
    // the weight fragments are re-read from cache each step: an opaque copy
    // of the pointer keeps the compiler from hoisting every fragment of every
    // layer into registers for the whole loop (which only spills them).  Up
    // to width 64 the copy stays a global-memory pointer, so the loads remain
    // global loads (through a generic pointer they are flat loads, which also
    // hold up every wait for LDS results); at width 128 the generic form
    // needs fewer registers and spills less
    const typename T::felem* fr = frag;
    if constexpr (W <= 64) {
      using gfelem = __attribute__((address_space(1))) const typename T::felem;
      gfelem* frg = (gfelem*)frag;
      asm volatile("" : "+s"(frg));
      fr = (const typename T::felem*)frg;
    } else {
      asm volatile("" : "+s"(fr));
    }
    float z[TPW][DIM], gv[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int64_t p = step * NB + col[t];
      bool interior = false;
      float fac = 0.f;
      const bool valid = p < total;
      if (valid) node_z<DIM>(p, geo.n, geo.ne, geo.bfac, z[t], &interior, &fac);
      else
        for (int c = 0; c < DIM; ++c) z[t][c] = 0.f;
      // the adjoint's loads first: their latency hides behind the recompute
      int64_t iq = -1;
      gv[t] = valid ? adjoint_at<float, DIM>(geo, qg, alpha, p, &iq) : 0.f;
      if (q == 0 && iq >= 0) lacc += res[iq] * qg[iq];
      if (obs_w && iq >= 0) {
        // data misfit w (u - d)^2 of the inverse problem (interior nodes)
        const float ow = obs_w[p], r = u[p] - obs_d[p];
        gv[t] += 2.f * ow * r;
        if (q == 0) lacc += ow * r * r;
      }
      if (geo.bfac) gv[t] *= fac;  // dLOSS/dNN = f dLOSS/du
    }
    float d[TPW][NR];
    forward_tiles<W, L, MODE, DIM, (W <= 64), TPW>(sp, fr, l1, z, q, lane, d, sink);
    if (q == 0) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        Gs[col[t]] = gv[t];
#pragma unroll
        for (int c = 0; c < DIM; ++c) Zs[c][col[t]] = z[t][c];
      }
    }
    // h_L through Dt for the output layer; then delta_L = g w_out (1 - h_L^2)
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int r = 0; r < NR; r += 2) {
        const int f0 = cfeat(r, q), f1 = cfeat(r + 1, q);
        T::lds_put2(Dt + f0 * LD + col[t], Dt + f1 * LD + col[t], DPL, d[t][r], d[t][r + 1]);
        d[t][r] = gv[t] * wo[f0] * (1.f - d[t][r] * d[t][r]);
        d[t][r + 1] = gv[t] * wo[f1] * (1.f - d[t][r + 1] * d[t][r + 1]);
      }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < FPT; ++f) {
      const int fq = (tid >> 2) + f * (NTH / 4);
      if (fq < W) {
        const E* hr = Dt + fq * LD + q4 * QN;
        float s = 0.f;
        for (int k = 0; k < QN; ++k) s += T::lds_get(hr + k, DPL) * Gs[q4 * QN + k];
        s_wout[f] += s;
      }
    }
    if (tid < 4) {
      float s = 0.f;
      for (int k = 0; k < QN; ++k) s += Gs[tid * QN + k];
      s_bout += s;
    }
    if constexpr (ND == 1) __syncthreads();
#pragma unroll
    for (int l = L; l >= 1; --l) {
      if constexpr (ND == 2) {
        ub ^= 1;
        Dt = Dts[ub];
      }
      // delta_l into Dt; for l >= 2 as the split operands the chain below uses
      typename T::op bop[TPW][NKS];
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        if (l >= 2) {
#pragma unroll
          for (int ks = 0; ks < NKS; ++ks) {
            bop[t][ks] = T::from(&d[t][ks * T::S]);
#pragma unroll
            for (int v = 0; v < T::S; ++v)
              T::lds_put_elem(Dt + cfeat(ks * T::S + v, q) * LD + col[t], DPL, bop[t][ks], v);
          }
        } else {
#pragma unroll
          for (int r = 0; r < NR; r += 2)
            T::lds_put2(Dt + cfeat(r, q) * LD + col[t], Dt + cfeat(r + 1, q) * LD + col[t], DPL, d[t][r],
                        d[t][r + 1]);
        }
      }
      __syncthreads();
      if (l >= 2) {
        // dW_l[o][i] += sum_nodes delta_l[o][node] h_{l-1}[i][node]
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
          const int tileid = w * OWN + o;
          if (tileid < NOB) {
            const int ob = tileid / NMB, ib = tileid % NMB;
            const E* arow = Dt + (ob * 16 + n) * LD + T::S * q;
            const E* brow = Hall + ((l - 2) * W + ib * 16 + n) * LD + T::S * q;
#pragma unroll
            for (int ks = 0; ks < NB / T::KS; ++ks) {
              const typename T::op av = T::lds_op(arow + ks * T::KS, DPL);
              acc[l - 2][o] = T::mma(av, T::lds_op(brow + ks * T::KS, HPL), acc[l - 2][o]);
              // db_l = delta_l times a ones column, once per output row block
              if (ib == 0) bacc[l - 2][o / NMB] = T::row_sum(av, bacc[l - 2][o / NMB]);
            }
          }
        }
      }
      // layer 1: db_1[f] = sum_n delta_1[f][n], dW_1[f][c] = sum_n delta_1[f][n] z_c[n]
#pragma unroll
      for (int f = 0; f < FPT; ++f) {
        const int fq = (tid >> 2) + f * (NTH / 4);
        if (l == 1 && fq < W) {
          const E* dr = Dt + fq * LD + q4 * QN;
          float sb = 0.f;
          float sw[DIM];
#pragma unroll
          for (int c = 0; c < DIM; ++c) sw[c] = 0.f;
          for (int k = 0; k < QN; ++k) {
            const float dv = T::lds_get(dr + k, DPL);
            sb += dv;
#pragma unroll
            for (int c = 0; c < DIM; ++c) sw[c] += dv * Zs[c][q4 * QN + k];
          }
          s_b[0][f] += sb;
#pragma unroll
          for (int c = 0; c < DIM; ++c) s_w1[c][f] += sw[c];
        }
      }
      if (l >= 2) {
        // delta_{l-1} = (W_l^T delta_l) (1 - h_{l-1}^2), one fragment load for all tiles
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
          f32x4_t c2[TPW];
#pragma unroll
          for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) c2[t][i] = 0.f;
#pragma unroll
          for (int ks = 0; ks < NKS; ++ks) {
            const auto f = T::frag(fr + frag_index<MODE>(l - 2, 1, mb, ks, lane, 0, W));
#pragma unroll
            for (int t = 0; t < TPW; ++t) c2[t] = T::mma_w(f, bop[t][ks], c2[t]);
          }
#pragma unroll
          for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float hv =
                  T::lds_get(Hall + ((l - 2) * W + cfeat(mb * 4 + i, q)) * LD + col[t], HPL);
              d[t][mb * 4 + i] = c2[t][i] * (1.f - hv * hv);
            }
        }
      }
      if constexpr (ND == 1) __syncthreads();  // Dt (and Hall in the next step) are rewritten
    }
    if constexpr (ND == 2) {
      ub ^= 1;
      gb ^= 1;
    }
  }
  // ---- this block's partial gradient row ----
  float* row = partials + int64_t(blockIdx.x) * ldp;
#pragma unroll
  for (int l = 2; l <= L; ++l) {
    const int64_t off = off_layer(l, DIM, W);
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
      const int tileid = w * OWN + o;
      if (tileid < NOB) {
        const int ob = tileid / NMB, ib = tileid % NMB;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int orow = ob * 16 + 4 * q + i;
          row[off + int64_t(orow) * W + ib * 16 + n] = acc[l - 2][o][i];
          if (ib == 0 && n == 0) row[off + int64_t(W) * W + orow] = bacc[l - 2][o / NMB][i];
        }
      }
    }
  }
  // small gradients: add the four node quarters of each feature through LDS
  auto reduce4 = [&](float v, int64_t dst, bool ok) {
    Red[tid] = v;
    __syncthreads();
    if (ok && q4 == 0) row[dst] = ((Red[tid] + Red[tid + 1]) + Red[tid + 2]) + Red[tid + 3];
    __syncthreads();
  };
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    const int fq = (tid >> 2) + f * (NTH / 4);
    const bool ok = fq < W;
    reduce4(s_wout[f], off_layer(L + 1, DIM, W) + fq, ok);
    reduce4(s_b[0][f], off_layer(1, DIM, W) + int64_t(W) * DIM + fq, ok);
#pragma unroll
    for (int c = 0; c < DIM; ++c) reduce4(s_w1[c][f], int64_t(fq) * DIM + c, ok);
  }
  Red[tid] = (tid < 4) ? s_bout : 0.f;  // threads 0..3 summed one node quarter of g each
  __syncthreads();
  if (tid == 0) row[off_layer(L + 1, DIM, W) + W] = ((Red[0] + Red[1]) + Red[2]) + Red[3];
  __syncthreads();
  const float lt = block_sum_n<NTH>(lacc, Red);
  if (tid == 0) loss_part[blockIdx.x] = lt;
}

// ---------------------------------------------------------------------------
// Fused gradient reduction + Adam + fragment update.  Partial rows have pitch
// ldp (a multiple of 4 floats).  Block = RW waves over 4 RC parameters: lane
// (c = lane % RC, g = lane / RC) of wave w reads parameters 4c..4c+3 (one
// 16-byte load) of rows (64/RC) w + g, then every (64/RC) RW rows further;
// the per-thread sums are added in a fixed order (RC = 16: 64 parameters
// per block; 32 per block measured slower, its final sum twice as long).
// The updated weight of a hidden-to-hidden layer is written straight
// into its two fragment slots.  One extra block sums the iteration's loss
// partials.
// ---------------------------------------------------------------------------
constexpr int RW = 16;  // waves per reduction block
constexpr int RC = 16;  // 16-byte column groups per reduction block

template <int MODE>
__device__ inline void adam_one(int64_t p, float gg, float* __restrict__ th, float* __restrict__ m,
                                float* __restrict__ v, float lr, float b1, float b2, float eps,
                                float c1, float c2, int dim, int W, int hidden,
                                typename MM<MODE>::felem* __restrict__ frag) {
  using T = MM<MODE>;
  const float mm = b1 * m[p] + (1.f - b1) * gg;
  const float vv = b2 * v[p] + (1.f - b2) * gg * gg;
  m[p] = mm;
  v[p] = vv;
  const float nw = th[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  th[p] = nw;
  // hidden-to-hidden weight? layer l = 2..hidden occupies [off_l, off_l + W*W)
  // (parameter counts are far below 2^31: 32-bit index arithmetic)
  const int base = W * dim + W;
  if (p < base) return;
  const int rel = int(p) - base, per = W * W + W;
  const int hl = rel / per;
  const int within = rel - hl * per;
  if (hl >= hidden - 1 || within >= W * W) return;
  const int o = within / W, i = within - o * W;
  int tt, qq;
  cfeat_inv(i, &tt, &qq);  // forward fragment (scaled): row o, contraction feature i
  T::put(frag + frag_index<MODE>(hl, 0, o >> 4, tt / T::S, (o & 15) + 16 * qq, tt % T::S, W),
         kTanhScale * nw);
  cfeat_inv(o, &tt, &qq);  // backward fragment: row i, contraction feature o
  T::put(frag + frag_index<MODE>(hl, 1, i >> 4, tt / T::S, (i & 15) + 16 * qq, tt % T::S, W), nw);
}

template <int MODE>
__global__ __launch_bounds__(64 * RW) void k_reduce_adam_pack(
    const float* __restrict__ part, int rows, int64_t P, int64_t ldp, float* __restrict__ th,
    float* __restrict__ m, float* __restrict__ v, double lr, double b1, double b2, double eps,
    const long long* __restrict__ t_dev, int dim, int W, int hidden,
    typename MM<MODE>::felem* __restrict__ frag, const float* __restrict__ loss_part, int loss_np,
    double* __restrict__ hist, int cap, int64_t zb) {
  part = zofs(part, zb); th = zofs(th, zb); m = zofs(m, zb); v = zofs(v, zb);
  t_dev = zofs(t_dev, zb); frag = zofs(frag, zb); loss_part = zofs(loss_part, zb);
  hist = zofs(hist, zb);
  constexpr int RG = 64 / RC;   // row groups per wave
  constexpr int RS = RG * RW;   // row stride of a thread
  __shared__ f32x4_t red[RS][RC];
  if (blockIdx.x == gridDim.x - 1) {
    __shared__ double lb[64 * RW];
    double s = 0;
    for (int k = threadIdx.x; k < loss_np; k += 64 * RW) s += double(loss_part[k]);
    const double tot = block_sum(s, lb);
    if (threadIdx.x == 0) hist[(*t_dev - 1) % cap] = tot;
    return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, c = lane % RC, rg = lane / RC;
  const int64_t p0 = int64_t(blockIdx.x) * (4 * RC) + 4 * c;
  f32x4_t s = {0.f, 0.f, 0.f, 0.f};
  if (p0 < P) {
    const float* col = part + p0;
    int r = RG * w + rg;
    for (; r + 3 * RS < rows; r += 4 * RS) {
      const f32x4_t a0 = *reinterpret_cast<const f32x4_t*>(col + int64_t(r) * ldp);
      const f32x4_t a1 = *reinterpret_cast<const f32x4_t*>(col + int64_t(r + RS) * ldp);
      const f32x4_t a2 = *reinterpret_cast<const f32x4_t*>(col + int64_t(r + 2 * RS) * ldp);
      const f32x4_t a3 = *reinterpret_cast<const f32x4_t*>(col + int64_t(r + 3 * RS) * ldp);
      s += a0;
      s += a1;
      s += a2;
      s += a3;
    }
    for (; r < rows; r += RS) s += *reinterpret_cast<const f32x4_t*>(col + int64_t(r) * ldp);
  }
  red[RG * w + rg][c] = s;
  __syncthreads();
  // wave 0: one parameter per lane (lane = 4 c + component)
  const int64_t p = int64_t(blockIdx.x) * (4 * RC) + lane;
  if (w != 0 || lane >= 4 * RC || p >= P) return;
  const float* rf = reinterpret_cast<const float*>(&red[0][0]);
  float gg = rf[lane];
#pragma unroll 8
  for (int k = 1; k < RS; ++k) gg += rf[k * (4 * RC) + lane];
  const double t = double(*t_dev);
  const float c1 = float(1.0 - pow(b1, t)), c2 = float(1.0 - pow(b2, t));
  adam_one<MODE>(p, gg, th, m, v, float(lr), float(b1), float(b2), float(eps), c1, c2, dim, W,
                 hidden, frag);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
bool mlp_mfma_supported(int dim, int width, int hidden, int mode) {
  if (dim == 3 ? hidden != 4 : (dim != 2 || !(hidden == 3 || hidden == 4))) return false;
  if (mode == NET_BF16 || mode == NET_MIX || mode == NET_F32)
    return width == 32 || width == 64 || width == 128;
  return width == 32 || width == 64;
}

int64_t mlp_fragment_bytes(int width, int hidden) {
  return 2 * int64_t(width) * width * (hidden - 1) * 4;  // float32, or a bf16 hi/lo pair
}

void launch_pack_fragments(const float* theta, int dim, int width, int hidden, int mode,
                           void* frag, hipStream_t st) {
  if (mode == NET_MIX) mode = NET_X3;  // same fragments
  const int64_t total = 2 * int64_t(width) * width * (hidden - 1);
  if (total <= 0) return;
  const int blocks = cdiv(total, 256);
  if (mode == NET_F32)
    k_pack_fragments<NET_F32><<<blocks, 256, 0, st>>>(theta, dim, width, hidden, static_cast<float*>(frag));
  else if (mode == NET_BF16)
    k_pack_fragments<NET_BF16><<<blocks, 256, 0, st>>>(theta, dim, width, hidden, static_cast<__bf16*>(frag));
  else
    k_pack_fragments<NET_X3><<<blocks, 256, 0, st>>>(theta, dim, width, hidden, static_cast<__bf16*>(frag));
}

void launch_reduce_adam_pack(const float* partials, int rows, int64_t P, int64_t ldp, float* theta,
                             float* m, float* v, double lr, double b1, double b2, double eps,
                             const long long* t_dev, int dim, int width, int hidden, int mode,
                             void* frag, const float* loss_part, int loss_np, double* loss_hist,
                             int cap, hipStream_t st, Batch bz) {
  const dim3 blocks(cdiv(P, 4 * RC) + 1, 1, bz.n);
  if (mode == NET_MIX) mode = NET_X3;  // same fragments
#define CRV_RA(MM_, TT)                                                                           \
  k_reduce_adam_pack<MM_><<<blocks, 64 * RW, 0, st>>>(partials, rows, P, ldp, theta, m, v, lr, b1, b2, eps, \
                                                  t_dev, dim, width, hidden, static_cast<TT*>(frag), \
                                                  loss_part, loss_np, loss_hist, cap, bz.zb)
  if (mode == NET_F32) CRV_RA(NET_F32, float);
  else if (mode == NET_BF16) CRV_RA(NET_BF16, __bf16);
  else CRV_RA(NET_X3, __bf16);
#undef CRV_RA
}

template <int W, int L, int MODE>
static void fwd_inst(const Geom& g, const float* th, const void* frag, float* u, long long* tb,
                     hipStream_t st, Batch bz) {
  const int64_t total = ipow(g.n, g.dim);
  const int64_t tiles = (total + 15) / 16;
  const auto* fr = static_cast<const typename MM<MODE>::felem*>(frag);
  const dim3 grid(cdiv(tiles, 4 * fwd_tpw<W>()), 1, bz.n);
  if constexpr (L == 4) {
    if (g.dim == 3) {
      k_mlp_fwd_mfma<W, L, MODE, 3><<<grid, 256, 0, st>>>(g, th, fr, u, tb, bz.zb);
      return;
    }
  }
  k_mlp_fwd_mfma<W, L, MODE, 2><<<grid, 256, 0, st>>>(g, th, fr, u, tb, bz.zb);
}

// instantiated shapes: the forward of the mixed form is the split-bf16 one;
// the split-bf16 backward keeps two LDS planes and stops at width 64
#define CRV_FWD_SHAPES(X)                                                                    \
  X(32, 3, NET_F32) X(64, 3, NET_F32) X(128, 3, NET_F32) X(32, 4, NET_F32) X(64, 4, NET_F32)  \
  X(128, 4, NET_F32)                                                                         \
  X(32, 3, NET_BF16) X(64, 3, NET_BF16) X(128, 3, NET_BF16) X(32, 4, NET_BF16)                \
  X(64, 4, NET_BF16) X(128, 4, NET_BF16)                                                     \
  X(32, 3, NET_X3) X(64, 3, NET_X3) X(128, 3, NET_X3) X(32, 4, NET_X3) X(64, 4, NET_X3)       \
  X(128, 4, NET_X3)
#define CRV_BWD_SHAPES(X)                                                                    \
  X(32, 3, NET_F32) X(64, 3, NET_F32) X(128, 3, NET_F32) X(32, 4, NET_F32) X(64, 4, NET_F32)  \
  X(128, 4, NET_F32)                                                                         \
  X(32, 3, NET_BF16) X(64, 3, NET_BF16) X(128, 3, NET_BF16) X(32, 4, NET_BF16)                \
  X(64, 4, NET_BF16) X(128, 4, NET_BF16)                                                     \
  X(32, 3, NET_X3) X(64, 3, NET_X3) X(32, 4, NET_X3) X(64, 4, NET_X3)                        \
  X(32, 3, NET_MIX) X(64, 3, NET_MIX) X(128, 3, NET_MIX) X(32, 4, NET_MIX) X(64, 4, NET_MIX)  \
  X(128, 4, NET_MIX)

void launch_mlp_forward_mfma(const Geom& g, int width, int hidden, int mode, const float* theta,
                             const void* frag, float* u, long long* t_bump, hipStream_t st,
                             Batch bz) {
  if (mode == NET_MIX) mode = NET_X3;  // the forward of the mixed form is split bf16
#define CRV_FW(WW, LL, MM_) \
  if (width == WW && hidden == LL && mode == MM_) return fwd_inst<WW, LL, MM_>(g, theta, frag, u, t_bump, st, bz);
  CRV_FWD_SHAPES(CRV_FW)
#undef CRV_FW
}

// waves per backward block: 4 (64 nodes per block step); width 128 takes 8
// so that its weight-gradient tiles spread over more waves
// (6 waves for the mixed form at width 64, two blocks per CU, measured 1.6x
// slower than 4 waves at three blocks per CU)
// (float32 at width 128: 4 waves, the LDS of its activations, 139 KB, allows
// one block per CU)
constexpr int bwd_nw(int width, int mode) { return (width >= 128 && mode != NET_F32) ? 8 : 4; }

// 16-node tiles per wave: two for the plain-bf16 and mixed backward at width
// 64 in 2D (two blocks per CU of two waves per SIMD, each wave with two
// independent chains and one fragment load per two products), one otherwise
constexpr int bwd_tpw(int width, int mode, int dim) {
  return (width == 64 && dim == 2 && (mode == NET_BF16 || mode == NET_MIX)) ? 2 : 1;
}

// resident blocks per CU that the LDS of one block allows (160 KB per CU)
template <int W, int L, int MODE, int DIM>
static int bwd_lds_blocks() {
  const size_t lds =
      BwdShape<W, L, MODE, DIM, bwd_nw(W, MODE), bwd_tpw(W, MODE, DIM)>::lds_bytes();
  return int(std::max<size_t>(1, std::min<size_t>(4, (160u * 1024u) / lds)));
}

// blocks per CU: what the LDS allows, capped by the occupancy the compiled
// kernel reaches (registers) when a device is present
template <int W, int L, int MODE>
static int bwd_per_cu(int dim, bool query) {
  constexpr int NW = bwd_nw(W, MODE);
  int lds_blocks = 1, occ = 0;
  hipError_t e = hipSuccess;
  if (dim == 3) {
    if constexpr (L == 4) {
      lds_blocks = bwd_lds_blocks<W, L, MODE, 3>();
      if (query)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, k_mlp_bwd_mfma<W, L, MODE, 3, NW, bwd_tpw(W, MODE, 3)>, 64 * NW, 0);
    }
  } else {
    lds_blocks = bwd_lds_blocks<W, L, MODE, 2>();
    if (query)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &occ, k_mlp_bwd_mfma<W, L, MODE, 2, NW, bwd_tpw(W, MODE, 2)>, 64 * NW, 0);
  }
  if (!query) return lds_blocks;
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return std::max(1, std::min(lds_blocks, occ));
}

int mlp_bwd_mfma_blocks(const Geom& g, int width, int hidden, int mode, int cu_count,
                        bool query) {
  int per_cu = 1;
  const int nw = bwd_nw(width, mode);
#define CRV_BB(WW, LL, MM_) \
  if (width == WW && hidden == LL && mode == MM_) per_cu = bwd_per_cu<WW, LL, MM_>(g.dim, query);
  CRV_BWD_SHAPES(CRV_BB)
#undef CRV_BB
  const int64_t total = ipow(g.n, g.dim);
  const int nb = 16 * nw * bwd_tpw(width, mode, g.dim);
  const int64_t steps = (total + nb - 1) / nb;
  return int(std::max<int64_t>(1, std::min<int64_t>(steps, int64_t(cu_count) * per_cu)));
}

template <int W, int L, int MODE>
static void bwd_inst(const Geom& g, int64_t ldp, const float* th, const void* frag, const float* q,
                     const float* alpha, const float* res, float* partials, float* loss_part,
                     int blocks, hipStream_t st, Batch bz, const float* ow, const float* od,
                     const float* u) {
  constexpr int NW = bwd_nw(W, MODE);
  const auto* fr = static_cast<const typename MM<MODE>::felem*>(frag);
  const dim3 grid(blocks, 1, bz.n);
  if constexpr (L == 4) {
    if (g.dim == 3) {
      k_mlp_bwd_mfma<W, L, MODE, 3, NW, bwd_tpw(W, MODE, 3)><<<grid, 64 * NW, 0, st>>>(
          g, ldp, th, fr, q, alpha, res, partials, loss_part, bz.zb, ow, od, u);
      return;
    }
  }
  k_mlp_bwd_mfma<W, L, MODE, 2, NW, bwd_tpw(W, MODE, 2)><<<grid, 64 * NW, 0, st>>>(
      g, ldp, th, fr, q, alpha, res, partials, loss_part, bz.zb, ow, od, u);
}

void launch_mlp_backward_mfma(const Geom& g, int width, int hidden, int mode, int64_t ldp,
                              const float* theta, const void* frag, const float* q,
                              const float* alpha, const float* res, float* partials,
                              float* loss_part, int blocks, hipStream_t st, Batch bz,
                              const float* obs_w, const float* obs_d, const float* u) {
#define CRV_BW(WW, LL, MM_) \
  if (width == WW && hidden == LL && mode == MM_) \
    return bwd_inst<WW, LL, MM_>(g, ldp, theta, frag, q, alpha, res, partials, loss_part, blocks, \
                                 st, bz, obs_w, obs_d, u);
  CRV_BWD_SHAPES(CRV_BW)
#undef CRV_BW
}

}  // namespace crv
