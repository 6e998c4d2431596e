// crv_gram_solve_noalloc: the Gram solve q = G^-1 res of crv_gram_solve
// (eq. 26-28, 2D) on caller-owned device arrays, with no device allocation
// and no context.  Every table and work array it needs lives in one
// file-scope device array (`scratch`) of fixed size, which each GPU the
// library runs on holds until the process ends.  The call only enqueues
// kernels on the given stream: it can be captured in a HIP graph and used
// where hipMalloc is not allowed.
//
// Same arithmetic as the context path: the orthonormal DST-I basis (float64
// values rounded to float32, in matrix-core operand order) along y, the
// shifted tridiagonal lines T + lambda_k I along x factored in float64 on
// the device, and the inverse DST-I along y; the interior arrays padded to a
// pitch that is a multiple of 64.
#include <atomic>

#include "../../include/crv.h"
#include "kernels.h"

namespace crv {

crv_status report(crv_status s, const char* msg);  // runtime.cpp: crv_last_error

namespace {

constexpr int kMaxElem = 512;                     // n_elem limit of the call
constexpr int kMaxPitch = (kMaxElem - 1 + 63) / 64 * 64;  // 512
constexpr size_t kPlane = size_t(kMaxPitch) * kMaxPitch;  // floats per padded array
constexpr int kMaxDevices = 64;

// float arrays: packed basis, padded res, two work arrays, padded q, line
// factors (lt, 1/d); then float64 shifts and loss partials
constexpr size_t kFloats = 7 * kPlane;
constexpr size_t kBytes = kFloats * sizeof(float) + size_t(kMaxPitch) * sizeof(double) +
                          size_t(kMaxPitch) * sizeof(double);

__device__ __align__(256) char scratch[kBytes];

std::atomic<void*> g_scratch[kMaxDevices];

// the device address of this device's copy of `scratch` (looked up once per
// device with that device current; the array's host-side name is not a
// device address)
crv_status scratch_on_device(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return report(CRV_EHIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return report(CRV_EINVAL, "device index out of range");
  void* p = g_scratch[dev].load();
  if (!p) {
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return report(CRV_EHIP, "hipGetSymbolAddress(scratch) failed");
    g_scratch[dev].store(p);
  }
  *out = static_cast<char*>(p);
  return CRV_OK;
}

// the orthonormal DST-I basis S[k][j] = sqrt(2/(m+1)) sin((k+1)(j+1) pi/(m+1))
// (zero outside m x m), written straight into the matrix-core operand order of
// the products (row block mb of 32, K chunk kc of 16, lane, 8 values), and
// the line shifts lambda_k = 4 sin^2((k+1) pi / (2(m+1)))
__global__ void k_na_tables(int m, int mp, float* __restrict__ pk, double* __restrict__ shifts) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const double pi = 3.14159265358979323846;
  if (idx < mp) {
    const double sn = sin(double(idx + 1) * pi / (2.0 * (m + 1)));
    shifts[idx] = idx < m ? 4.0 * sn * sn : 2.0;
  }
  if (idx >= int64_t(mp) * mp) return;
  const int u = int(idx & 7), lane = int((idx >> 3) & 63);
  const int64_t chunk = idx >> 9;  // (mb, kc)
  const int kcs = mp / 16;
  const int mb = int(chunk / kcs), kc = int(chunk % kcs);
  const int row = 32 * mb + (lane & 31), col = 16 * kc + 2 * u + (lane >> 5);
  double v = 0.0;
  if (row < m && col < m)
    v = sqrt(2.0 / (m + 1)) * sin(double(row + 1) * double(col + 1) * pi / double(m + 1));
  pk[idx] = float(v);
}

// res (m x m, x fastest) into the zero-padded pitch-mp array; the line
// solve's output array cleared (the solve writes only its m x m part, and
// the rows beyond m enter the inverse product with zero weights, which an
// earlier call's non-finite leftovers would turn into NaN)
__global__ void k_na_pad(int m, int mp, const float* __restrict__ res, float* __restrict__ out,
                         float* __restrict__ cleared) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(mp) * mp) return;
  const int i = int(idx % mp), j = int(idx / mp);
  out[idx] = (i < m && j < m) ? res[int64_t(j) * m + i] : 0.f;
  cleared[idx] = 0.f;
}

// q out of the padded array; one block per row j also sums res.q of the row
// (fixed order) into part[j]
__global__ __launch_bounds__(256) void k_na_unpad_dot(int m, int mp, const float* __restrict__ qp,
                                                      const float* __restrict__ res,
                                                      float* __restrict__ q,
                                                      double* __restrict__ part) {
  __shared__ double sb[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const float v = qp[int64_t(j) * mp + i];
    q[int64_t(j) * m + i] = v;
    s += double(res[int64_t(j) * m + i]) * double(v);
  }
  s = block_sum(s, sb);
  if (threadIdx.x == 0) part[j] = s;
}

__global__ __launch_bounds__(256) void k_na_loss(int m, const double* __restrict__ part,
                                                 double* __restrict__ loss) {
  __shared__ double sb[256];
  double s = 0.0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) s += part[j];
  s = block_sum(s, sb);
  if (threadIdx.x == 0) *loss = s;
}

}  // namespace
}  // namespace crv

using namespace crv;

extern "C" crv_status crv_gram_solve_noalloc(int n_elem, const float* d_res, float* d_q,
                                             double* d_loss, void* stream) {
  if (n_elem < 4 || n_elem > kMaxElem)
    return report(CRV_EINVAL, "crv_gram_solve_noalloc: n_elem must be in [4, 512] (the size of "
                              "its fixed scratch array)");
  if (!d_res || !d_q) return report(CRV_EINVAL, "crv_gram_solve_noalloc: NULL array");
  char* base = nullptr;
  crv_status s = scratch_on_device(&base);
  if (s) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int m = n_elem - 1, mp = (m + 63) / 64 * 64;
  float* f = reinterpret_cast<float*>(base);
  float* pk = f;
  float* rpad = f + kPlane;
  float* rhat = f + 2 * kPlane;
  float* qhat = f + 3 * kPlane;
  float* qpad = f + 4 * kPlane;
  float* lt = f + 5 * kPlane;
  float* invd = f + 6 * kPlane;
  double* shifts = reinterpret_cast<double*>(f + kFloats);
  double* part = shifts + kMaxPitch;
  const int64_t plane = int64_t(mp) * mp;
  // tables (they depend on n_elem only; rebuilt each call, so a call never
  // relies on what an earlier one left in the scratch array)
  k_na_tables<<<cdiv(plane, 256), 256, 0, st>>>(m, mp, pk, shifts);
  launch_factor_shifted<float>(shifts, m, m, mp, 1.0, lt, invd, st);
  k_na_pad<<<cdiv(plane, 256), 256, 0, st>>>(m, mp, d_res, rpad, qhat);
  // DST-I along y, shifted lines along x, inverse DST-I along y
  launch_gemm<float>(mp, mp, mp, nullptr, mp, rpad, mp, rhat, mp, st, pk);
  launch_band_rows<float>(rhat, qhat, m, m, mp, 1, lt, invd, mp, mp, st);
  launch_gemm<float>(mp, mp, mp, nullptr, mp, qhat, mp, qpad, mp, st, pk);
  k_na_unpad_dot<<<m, 256, 0, st>>>(m, mp, qpad, d_res, d_q, part);
  if (d_loss) k_na_loss<<<1, 256, 0, st>>>(m, part, d_loss);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return report(CRV_EHIP, hipGetErrorString(e));
  return CRV_OK;
}
