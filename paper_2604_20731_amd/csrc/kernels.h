// Launchers of the libcrv HIP kernels (instantiated for float and double).
#pragma once
#include "common.h"

namespace crv {

// ---- fields (k_fields.hip) ------------------------------------------------
// a1: saturation at the nodes from the spline coefficients (knot values) and
// alpha = K (kr_w/mu_w + kr_g/mu_g) at clamp(S,0,1); flux (nullable) receives
// the buoyancy flux F = K (kr_w rho_w/mu_w + kr_g rho_g/mu_g).
template <typename Real>
void launch_refresh(const Geom& g, const Real* s_coefs, const int* knot_first, const Real* knot_val,
                    const Real* perm, double mu_w, double mu_g, double nexp, double rho_w,
                    double rho_g, Real* s_nodal, Real* alpha, Real* flux, hipStream_t st,
                    Batch bz = Batch{});
// pressure right-hand side with gravity (g = -gravity e_v, e_v = y in 2D, z in
// 3D): hq = h^d (qi + qp) + gravity h^(d-1) (F_{p+e_v} - F_p)
template <typename Real>
void launch_gravity_rhs(const Geom& g, const Real* flux, const Real* qi, const Real* qp,
                        double gravity, Real* hq, hipStream_t st, Batch bz = Batch{});

// a3: RES on the interior nodes (padded layout, pitch mp).
template <typename Real>
void launch_residual(const Geom& g, const Real* u, const Real* alpha, const Real* hq, Real* res,
                     hipStream_t st, Batch bz = Batch{});

// a5: g_u = 2 A^T q (zero on the boundary) and per-block partial sums of RES.q.
// With observations (obs_w non-null; obs_d the data, u the network pressure)
// 2 w (u - d) joins g_u and w (u - d)^2 the loss at interior nodes.
// Returns the number of partials written.
template <typename Real>
int launch_adjoint(const Geom& g, const Real* q, const Real* alpha, const Real* res, Real* gu,
                   Real* loss_partials, hipStream_t st, const Real* obs_w = nullptr,
                   const Real* obs_d = nullptr, const Real* u = nullptr);
// Adam step on the nodal log K (moments m, v, step count *t) and K = exp(log K)
template <typename Real>
void launch_adam_logk(int64_t n, Real* logk, Real* m, Real* v, const Real* g, Real* perm,
                      double lr, double b1, double b2, double eps, const long long* t,
                      hipStream_t st);
int adjoint_partials(const Geom& g);

// Sum of the loss partials (fixed order) into loss_hist[(t + slot_offset) % cap].
template <typename Real>
void launch_loss_finalize(const Real* partials, int np, double* loss_hist, int cap,
                          const long long* t_dev, int slot_offset, hipStream_t st);
// ++*t (one thread)
void launch_bump(long long* t, hipStream_t st);

// a3 differentiation form: dLOSS/dlogK = 2 sum_dir grad+ u . grad+ q h^(d-2) * alpha,
// with gravity (flux non-null) - 2 gravity h^(d-1) F_p (q_{p-e_v} - q_p).
template <typename Real>
void launch_grad_logperm(const Geom& g, const Real* u, const Real* q, const Real* alpha,
                         const Real* flux, double gravity, Real* out, hipStream_t st);

// a8: b_kl = int I_h(u) B_kl (Q1 nodal interpolant, exact Gauss).
template <typename Real>
void launch_project(const Geom& g, const Real* u, const Real* proj_val, Real* b, hipStream_t st,
                    Batch bz = Batch{});

// a10: b_kl = int [S B_kl + tau/phi (-lambda_g K (grad p - rho_g g) . grad B_kl + q_g B_kl)];
// gshift = rho_g gravity is added to the vertical derivative of p (g = -gravity e_v);
// tau is read from device memory so a captured step serves any step length.
template <typename Real>
void launch_ads_assemble(const Geom& g, const Real* s, const Real* p, const Real* perm,
                         const Real* poro, const Real* qi, const Real* qp, const Real* gb,
                         const Real* gdb, const Real* gxi, const Real* gw, const double* tau,
                         double mu_w, double mu_g, double nexp, double gshift, Real* b,
                         hipStream_t st, Batch bz = Batch{});

// ---- IGA Galerkin pressure system, 2D (k_galerkin.hip; eq. 15-20) --------
// Device arrays of one solve (owned by the context): Gauss-point arrays
// (Ne (r+1))^2, coefficient arrays nb^2, 5 scalars and 2 x galerkin_partials
// partial sums.
template <typename Real>
struct GalerkinWork {
  Real *c, *f0, *fy;              // w alpha, w q, -gravity w F_b at the Gauss points
  Real *f, *dg, *r, *z, *p, *p2, *ap;  // load, diagonal, CG vectors (two direction arrays)
  double *sc, *part, *part2;       // scalars, operator tile partials, update-block pairs
  // Kronecker preconditioner: mg = nb - 2 interior coefficients per axis,
  // padded to mgp (a multiple of 64); ksc (nb^2) the diagonal scaling,
  // kt0..kt2 (mgp^2) work arrays, ksym (2 mgp) the 1D mass and stiffness
  // symbols, kdst (mgp^2, and packed) the orthonormal DST-I basis of size mg
  int mg, mgp;
  Real *ksc, *kt0, *kt1, *kt2, *ksym, *kdst, *kdst_pk;
};
// partial sums a solve writes at most (operator tiles or dot-product blocks)
int64_t galerkin_partials(const Geom& g);
template <typename Real>
struct GalerkinArgs {
  const Real *s, *perm, *qi, *qp, *gb, *gdb, *gxi, *gw;
  double mu_w, mu_g, nexp, rho_w, rho_g, gravity;
  Real* x;  // the solution (pressure coefficients; boundary coefficients 0)
  GalerkinWork<Real> ws;
  int precond;  // 0 diagonal of S, 1 scaled Kronecker inverse
};
// fields at the Gauss points, load, diagonal; x = 0 and the first CG vectors
template <typename Real>
void launch_galerkin_setup(const Geom& g, const GalerkinArgs<Real>& a, hipStream_t st);
// iters CG iterations from rz in slot 0 (they alternate the slot, so a
// further call continues correctly only after an even count; scalars stay on
// the device: sc[3] = r.r, sc[4] = F.F)
template <typename Real>
void launch_galerkin_iters(const Geom& g, const GalerkinArgs<Real>& a, int iters, hipStream_t st);
// r.r of the last update into sc[3] (the operator records it only at the
// start of the next iteration), after the last chunk
template <typename Real>
void launch_galerkin_finish(const GalerkinWork<Real>& w, hipStream_t st);

// K7f: float64 factorisations on the device.
// Banded LDL^T of the 1D mass matrix (band (nb, r+1)) -> lt (nb*r), inv_d (nb).
template <typename Real>
void launch_factor_band(const double* band, int n, int r, double* work_d, Real* lt, Real* inv_d,
                        int* status, hipStream_t st);
// LDL^T of the shifted tridiagonals scale*(T + shift_k I), T = tridiag(-1,2,-1)
// of size m; line k has shift shifts[k]; tables pitch mp.
template <typename Real>
void launch_factor_shifted(const double* shifts, int nlines, int m, int mp, double scale,
                           Real* lt, Real* inv_d, hipStream_t st);

// *p = v on the stream (device memory, no host synchronisation)
void launch_set_f64(double* p, double v, hipStream_t st);
// the same for n scenarios: *(p + k zb bytes) = v[k], k < n
void launch_set_f64_batch(double* p, int64_t zb, const double* v, int n, hipStream_t st);
template <typename Real>
void launch_fill(Real* p, size_t n, Real v, hipStream_t st);
template <typename Src, typename Dst>
void launch_convert(const Src* in, Dst* out, size_t n, hipStream_t st);
// logk[i] = src[i], perm[i] = exp(src[i]) (float32 contexts, src on the device)
void launch_set_logk(int64_t n, const float* src, float* logk, float* perm, hipStream_t st);
// non-finite check: sets *flag = 1 if any entry is NaN/Inf
template <typename Real>
void launch_check_finite(const Real* p, size_t n, int* flag, hipStream_t st, Batch bz = Batch{});

// ---- solves (k_solve.hip) --------------------------------------------------
// Banded unit-lower L D L^T solves along contiguous lines: one wavefront per
// line, chunked recurrence + wavefront affine scan.  Line l occupies
// x[l*line_stride + j], j < n.  Coefficients: lt[(l*coef_stride) + j*r + t-1]
// = L(j, j-t), inv_d[(l*coef_stride_d) + j].  In place allowed (x == b).
template <typename Real>
void launch_band_rows(const Real* b, Real* x, int n, int nlines, int64_t line_stride, int r,
                      const Real* lt, const Real* inv_d, int64_t coef_stride,
                      int64_t coef_stride_d, hipStream_t st, Batch bz = Batch{});
// Same solve along strided lines (element j of line c at x[j*row_stride + c]),
// shared coefficients, over batch planes batch_stride apart.  A scenario batch
// (2D passes only, batch = 1) takes the place of the planes.
template <typename Real>
void launch_band_cols(const Real* b, Real* x, int n, int nlines, int64_t row_stride, int r,
                      const Real* lt, const Real* inv_d, int64_t batch, int64_t batch_stride,
                      hipStream_t st, Batch bz = Batch{});

// C = A B, row-major, all dims multiples of 64, pitches in elements.
// a_packed (nullable, float32 only): A as packed matrix-core fragments
// (pack_gemm_a in tables.h), used instead of A when given.
template <typename Real>
void launch_gemm(int M, int N, int K, const Real* A, int lda, const Real* B, int ldb, Real* C,
                 int ldc, hipStream_t st, const Real* a_packed = nullptr);
// batch products sharing A: C_z = A B_z, B_z = B + z sb, C_z = C + z sc
template <typename Real>
void launch_gemm_batched(int M, int N, int K, const Real* A, int lda, const Real* B, int ldb,
                         int64_t sb, Real* C, int ldc, int64_t sc, int batch, hipStream_t st,
                         const Real* a_packed = nullptr);

// C = A B for square M x M operands (M a multiple of 64, leading dimensions M)
// with an epilogue: epi 0 stores C, 1 stores C^T, 2 stores
// C_ij / (sym[M+i] sym[j] + sym[i] sym[M+j]).  float needs a_packed (the
// call does nothing without it); double ignores it.  skip (nullable, device):
// the product is left out when skip[0] <= skip[3] at the time it runs.
template <typename Real>
void launch_gemm_sq_epi(int M, const Real* A, const Real* B, Real* C, int epi, const Real* sym,
                        hipStream_t st, const Real* a_packed, const double* skip);

// ---- network (k_mlp.hip) ---------------------------------------------------
struct MlpShape {
  int dim, width, hidden;
  int64_t nparams;
};
int64_t mlp_param_count(int dim, int width, int hidden);
// u = f * NN(2x-1) on all nodes (f the trial-function factor); t_bump (nullable) is incremented once.
template <typename Real>
void launch_mlp_forward(const Geom& g, const MlpShape& s, const Real* theta, Real* u,
                        long long* t_bump, hipStream_t st);
// per-block partial gradients of sum_p gu_p NN(z_p); returns rows written
template <typename Real>
int launch_mlp_backward(const Geom& g, const MlpShape& s, const Real* theta, const Real* gu,
                        Real* partials, hipStream_t st);
int mlp_backward_rows(const Geom& g, const MlpShape& s, int real_bytes);
// fixed-order column sums of partials (rows x P, row pitch ld) -> out (P); uses scratch
template <typename Real>
void launch_reduce_rows(const Real* in, int rows, int64_t P, int64_t ld, Real* scratch, Real* out,
                        hipStream_t st);
template <typename Real>
void launch_adam(int64_t P, Real* theta, Real* m, Real* v, const Real* g, double lr,
                 double beta1, double beta2, double eps, const long long* t_dev,
                 hipStream_t st);

// ---- network on matrix cores (k_mlp_mfma.hip), float32 parameters ----------
// arithmetic of the hidden-to-hidden products
// NET_MIX: split-bf16 forward (the pressure the loss sees), plain bf16
// backward products; its fragments are the split-bf16 ones
enum NetMode : int { NET_F32 = 0, NET_BF16 = 1, NET_X3 = 2, NET_MIX = 3 };
bool mlp_mfma_supported(int dim, int width, int hidden, int mode);
int64_t mlp_fragment_bytes(int width, int hidden);
// rearrange theta into the MFMA operand fragments of the mode
void launch_pack_fragments(const float* theta, int dim, int width, int hidden, int mode,
                           void* frag, hipStream_t st);
void launch_mlp_forward_mfma(const Geom& g, int width, int hidden, int mode, const float* theta,
                             const void* frag, float* u, long long* t_bump, hipStream_t st,
                             Batch bz = Batch{});
// backward blocks: at most cu_count x the blocks per CU that one block's LDS
// allows; with query, also capped by the occupancy the compiled kernel reaches
int mlp_bwd_mfma_blocks(const Geom& g, int width, int hidden, int mode, int cu_count, bool query);
// partial gradient rows (pitch ldp, a multiple of 4) of sum_p g_u(p) NN(z_p)
// with g_u = 2 A^T q evaluated per node from q and alpha; loss_part[block] =
// the block's share of RES . q
void launch_mlp_backward_mfma(const Geom& g, int width, int hidden, int mode, int64_t ldp,
                              const float* theta, const void* frag, const float* q,
                              const float* alpha, const float* res, float* partials,
                              float* loss_part, int blocks, hipStream_t st, Batch bz = Batch{},
                              const float* obs_w = nullptr, const float* obs_d = nullptr,
                              const float* u = nullptr);
// fixed-order sum of the partial rows + Adam + fragment update; one extra
// block sums the loss partials into loss_hist[(t-1) % cap]
void launch_reduce_adam_pack(const float* partials, int rows, int64_t P, int64_t ldp, float* theta, float* m,
                             float* v, double lr, double b1, double b2, double eps,
                             const long long* t_dev, int dim, int width, int hidden, int mode,
                             void* frag, const float* loss_part, int loss_np, double* loss_hist,
                             int cap, hipStream_t st, Batch bz = Batch{});

}  // namespace crv
