// Shared device/host helpers of libcrv (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace crv {

constexpr int kWave = 64;

// Geometry of one 2D/3D scenario.
struct Geom {
  int dim;  // 2 or 3
  int ne;   // elements per axis
  int n;    // nodes per axis (ne + 1)
  int r;    // B-spline degree
  int nb;   // coefficients per axis (ne + r)
  int m;    // interior nodes per axis (ne - 1)
  int mp;   // padded pitch of interior arrays (multiple of 64)
  int bfac = 0;  // trial-function factor: 0 interior indicator, 1 prod 4 x (1 - x)
};

// Scenario batching.  Scenarios of one configuration whose workspaces lie zb
// bytes apart advance with one launch per kernel: blockIdx.z selects the
// scenario and every pointer argument (an address in the first scenario's
// workspace) moves by blockIdx.z * zb bytes.  n = 1, zb = 0 is a single
// scenario.  Only kernels whose grid leaves z free take a batch.
struct Batch {
  int n = 1;
  int64_t zb = 0;
};

// (byte arithmetic on the pointer itself, not through an integer, so the
// compiler still knows a kernel argument's address points to global memory
// and emits global rather than flat loads: a flat load also counts as an
// LDS/scalar access, so every wait for one of those waited for it as well)
template <typename T>
__device__ inline T* zofs(T* p, int64_t zb) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p ? reinterpret_cast<T*>(reinterpret_cast<B*>(p) + int64_t(blockIdx.z) * zb) : p;
}
// the same through an integer: the address space is lost and the accesses are
// flat.  Kept for the forward network kernel's weight fragments, whose global
// loads the compiler hoists further, which costs the kernel a wave per SIMD
template <typename T>
__device__ inline T* zofs_flat(T* p, int64_t zb) {
  return p ? reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + uint64_t(blockIdx.z) * uint64_t(zb))
           : p;
}

__host__ __device__ inline int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// tanh from its definition 1 - 2/(exp(2x)+1), on the hardware base-2
// exponential and reciprocal (each about 1 ulp): exp(2x) = 2^(x * 2/ln 2).
// Overflow of the exponential gives +1, underflow -1.
__device__ inline float tanh_fast(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);
  return __builtin_fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}
__device__ inline double tanh_fast(double x) { return tanh(x); }

template <typename T>
__device__ inline T clamp01(T s) {
  return s < T(0) ? T(0) : (s > T(1) ? T(1) : s);
}

// s^n for the Brooks-Corey exponent; exact products for n = 1, 2, 3.
template <typename T>
__device__ inline T powi_or_pow(T s, T n) {
  if (n == T(2)) return s * s;
  if (n == T(1)) return s;
  if (n == T(3)) return s * s * s;
  return pow(s, n);
}

template <typename T>
__device__ inline T shfl_up(T v, int d) {
  return __shfl_up(v, d, kWave);
}
template <typename T>
__device__ inline T shfl_down(T v, int d) {
  return __shfl_down(v, d, kWave);
}
template <typename T>
__device__ inline T shfl(T v, int l) {
  return __shfl(v, l, kWave);
}

// Fixed-order block sum over blockDim.x <= 1024 threads (a block size that is
// not a power of two first folds its top part onto the first threads).
template <typename T>
__device__ inline T block_sum(T v, T* sbuf) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int p2 = 1 << (31 - __builtin_clz(nt));  // largest power of two <= nt
  sbuf[tid] = v;
  __syncthreads();
  if (tid < nt - p2) sbuf[tid] += sbuf[tid + p2];  // fold the rest (none when nt = p2)
  if (nt != p2) __syncthreads();
  for (int s = p2 / 2; s > 0; s >>= 1) {
    if (tid < s) sbuf[tid] += sbuf[tid + s];
    __syncthreads();
  }
  T out = sbuf[0];
  __syncthreads();
  return out;
}

// The same sum for a block of NT threads known at compile time (no fold code
// for a power of two).
template <int NT, typename T>
__device__ inline T block_sum_n(T v, T* sbuf) {
  constexpr int p2 = NT >= 512 ? 512 : NT >= 256 ? 256 : NT >= 128 ? 128 : 64;
  static_assert(NT <= 1023 && NT >= 64, "64 to 1023 threads");
  const int tid = threadIdx.x;
  sbuf[tid] = v;
  __syncthreads();
  if constexpr (NT != p2) {
    if (tid < NT - p2) sbuf[tid] += sbuf[tid + p2];
    __syncthreads();
  }
  for (int s = p2 / 2; s > 0; s >>= 1) {
    if (tid < s) sbuf[tid] += sbuf[tid + s];
    __syncthreads();
  }
  T out = sbuf[0];
  __syncthreads();
  return out;
}

inline int cdiv(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// a = q n + r for 0 <= a < 2^31 without an integer division: q from a float64
// product with 1/n (off by at most one near multiples of n), then corrected.
__device__ inline void divmod_u32(uint32_t a, uint32_t n, uint32_t* q, uint32_t* r) {
  uint32_t qq = uint32_t(double(a) * (1.0 / double(n)));
  int64_t rr = int64_t(a) - int64_t(qq) * n;
  if (rr < 0) {
    --qq;
    rr += n;
  } else if (rr >= int64_t(n)) {
    ++qq;
    rr -= n;
  }
  *q = qq;
  *r = uint32_t(rr);
}

// grid indices (i, j[, k]) of node p on n^dim nodes, x fastest (p < 2^31)
template <int DIM>
__device__ inline void node_ijk(int64_t p, int n, int* i, int* j, int* k) {
  uint32_t q1, r1;
  divmod_u32(uint32_t(p), uint32_t(n), &q1, &r1);
  *i = int(r1);
  if (DIM == 3) {
    uint32_t q2, r2;
    divmod_u32(q1, uint32_t(n), &q2, &r2);
    *j = int(r2);
    *k = int(q2);
  } else {
    *j = int(q1);
    *k = 0;
  }
}

// trial-function factor at an interior node (i, j[, k]) (eq. 23 asks only
// that the trial functions vanish on the boundary): 1 for the interior
// indicator, prod_a 4 x_a (1 - x_a), x_a = i_a / ne, for the distance form
// (float64, the axes multiplied in the order i, j, k)
template <int DIM>
__device__ inline double trial_factor(int bfac, int ne, int i, int j, int k) {
  if (!bfac) return 1.0;
  const double xi = double(i) / double(ne), xj = double(j) / double(ne);
  double f = (4.0 * xi * (1.0 - xi)) * (4.0 * xj * (1.0 - xj));
  if (DIM == 3) {
    const double xk = double(k) / double(ne);
    f *= 4.0 * xk * (1.0 - xk);
  }
  return f;
}

}  // namespace crv
