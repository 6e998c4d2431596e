// libcrv host runtime: the C ABI of include/crv.h.
//
// One context = one scenario on one device stream.  All state (fields,
// factor tables, network parameters, Adam moments, loss history) lives in a
// single device workspace carved at init; after init the coupled step runs
// entirely on the device and the host only reads results back on request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/crv.h"
#include "kernels.h"
#include "tables.h"

namespace crv {

static thread_local std::string g_err;

static crv_status fail(crv_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

// the same for the library's other translation units
crv_status report(crv_status s, const char* msg) { return fail(s, msg); }

#define CRV_HIP(x)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return fail(CRV_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kLossCap = 1 << 16;

// ---------------------------------------------------------------------------
// workspace layout (identical dry run for crv_workspace_size)
// ---------------------------------------------------------------------------
// Addresses are formed as integers: the sizing dry run carves from a null
// base, and pointer arithmetic on a null pointer is undefined.
struct Carve {
  uintptr_t base;
  size_t off = 0;
  explicit Carve(void* b) : base(reinterpret_cast<uintptr_t>(b)) {}
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += n * sizeof(T);
    return p;
  }
};

// Gram line solves: one tridiagonal line per interior (y[, z]) mode, padded
// modes included in 3D so that the line index is the row index of the array
static int64_t gram_lines(const Geom& g) { return g.dim == 3 ? int64_t(g.m) * g.mp : g.m; }

// pitch of the matrix-core backward's partial gradient rows: P rounded up to
// 32 floats, so every row starts on a 128-byte line and the reduction's
// 256-byte slices of a row touch two lines, not three
static int64_t partial_pitch(int64_t P) { return (P + 31) / 32 * 32; }

static Geom make_geom(const crv_config& c) {
  Geom g;
  g.dim = c.dim;
  g.ne = c.n_elem;
  g.n = c.n_elem + 1;
  g.r = c.degree;
  g.nb = c.n_elem + c.degree;
  g.m = c.n_elem - 1;
  g.mp = (g.m + 63) / 64 * 64;
  g.bfac = c.boundary_factor;
  return g;
}

template <typename Real>
struct Buffers {
  // nodal (N+1)^d
  Real *perm, *poro, *qi, *qp, *hq, *s_nodal, *alpha, *u, *gu, *tmp_nodal;
  Real* gflux;     // buoyancy flux K (kr_w rho_w/mu_w + kr_g rho_g/mu_g) (gravity only)
  // coefficients nb^d
  Real *s, *p, *bvec;
  // interior, padded to mp per axis
  Real *res, *rhat, *qhat, *q, *dst, *dst_pk;
  // Gram lines (pitch mp) and mass factors
  Real *g_lt, *g_invd, *m_lt, *m_invd;
  double *band, *band_work, *shifts;
  int* status;
  // tables
  int* knot_first;
  Real *knot_val, *proj_val, *gb, *gdb, *gxi, *gw;
  // network and optimiser
  Real *theta, *am, *av, *grad, *partials, *red_scratch, *loss_part;
  double *loss_hist, *loss_scalar;
  long long *t_dev, *t_zero;
  double* tau;     // substep length of the current step (device, read by the assembly)
  int* flag;
  // inverse problem: observation weights and data (nodal), log K and the
  // moments and step count of its Adam
  Real *obs_w, *obs_d, *logk, *lk_m, *lk_v;
  long long* t_k;
  void* frag;      // MFMA weight fragments (bf16 or float32)
  int bwd_rows;
  int loss_np;
};

constexpr int kMaxCUs = 256;  // compute units sized for (MI355X); persistent grids use at most this

static int net_mode(const crv_config& c) {
  return c.precision == CRV_PREC_BF16     ? NET_BF16
         : c.precision == CRV_PREC_BF16X3 ? NET_X3
         : c.precision == CRV_PREC_BF16X3F ? NET_MIX
                                           : NET_F32;
}

static bool uses_mfma(const crv_config& c) {
  return c.precision != CRV_PREC_FP64 && mlp_mfma_supported(c.dim, c.width, c.hidden, net_mode(c));
}

template <typename Real>
static size_t carve(Carve& cv, const crv_config& c, Buffers<Real>& b) {
  const Geom g = make_geom(c);
  const size_t nn = size_t(ipow(g.n, g.dim));
  const size_t nc = size_t(ipow(g.nb, g.dim));
  const size_t ni = size_t(ipow(g.mp, g.dim));
  const size_t nl = size_t(gram_lines(g));
  const int64_t P = mlp_param_count(c.dim, c.width, c.hidden);
  MlpShape ms{c.dim, c.width, c.hidden, P};
  b.perm = cv.take<Real>(nn);
  b.poro = cv.take<Real>(nn);
  b.qi = cv.take<Real>(nn);
  b.qp = cv.take<Real>(nn);
  b.hq = cv.take<Real>(nn);
  b.s_nodal = cv.take<Real>(nn);
  b.alpha = cv.take<Real>(nn);
  b.u = cv.take<Real>(nn);
  b.gu = cv.take<Real>(nn);
  b.tmp_nodal = cv.take<Real>(nn);
  b.gflux = cv.take<Real>(c.gravity != 0.0 ? nn : 0);
  b.s = cv.take<Real>(nc);
  b.p = cv.take<Real>(nc);
  b.bvec = cv.take<Real>(nc);
  b.res = cv.take<Real>(ni);
  b.rhat = cv.take<Real>(ni);
  b.qhat = cv.take<Real>(ni);
  b.q = cv.take<Real>(ni);
  b.dst = cv.take<Real>(size_t(g.mp) * g.mp);
  b.dst_pk = cv.take<Real>(size_t(g.mp) * g.mp);
  b.g_lt = cv.take<Real>(nl * g.mp);
  b.g_invd = cv.take<Real>(nl * g.mp);
  b.m_lt = cv.take<Real>(size_t(g.nb) * g.r);
  b.m_invd = cv.take<Real>(size_t(g.nb));
  b.band = cv.take<double>(size_t(g.nb) * (g.r + 1));
  b.band_work = cv.take<double>(size_t(g.nb) * (g.r + 1));
  b.shifts = cv.take<double>(nl);
  b.status = cv.take<int>(1);
  b.knot_first = cv.take<int>(size_t(g.n));
  b.knot_val = cv.take<Real>(size_t(g.n) * (g.r + 1));
  b.proj_val = cv.take<Real>(size_t(g.nb) * (g.r + 2));
  b.gb = cv.take<Real>(size_t(g.ne) * (g.r + 1) * (g.r + 1));
  b.gdb = cv.take<Real>(size_t(g.ne) * (g.r + 1) * (g.r + 1));
  b.gxi = cv.take<Real>(size_t(g.r + 1));
  b.gw = cv.take<Real>(size_t(g.r + 1));
  b.theta = cv.take<Real>(P);
  b.am = cv.take<Real>(P);
  b.av = cv.take<Real>(P);
  b.grad = cv.take<Real>(P);
  b.frag = cv.take<char>(size_t(std::max<int64_t>(4, mlp_fragment_bytes(c.width, c.hidden))));
  b.bwd_rows = uses_mfma(c) ? mlp_bwd_mfma_blocks(g, c.width, c.hidden, net_mode(c), kMaxCUs, false)
                            : mlp_backward_rows(g, ms, int(sizeof(Real)));
  b.partials = cv.take<Real>(size_t(b.bwd_rows) * partial_pitch(P));  // pitch ldp (MFMA) or P
  b.red_scratch = cv.take<Real>(size_t(2) * cdiv(b.bwd_rows, 64) * P);
  // loss partials: from the adjoint kernel, or one per fused network-backward block
  b.loss_np = std::max(adjoint_partials(g), b.bwd_rows);
  b.loss_part = cv.take<Real>(size_t(b.loss_np));
  b.loss_hist = cv.take<double>(kLossCap);
  b.loss_scalar = cv.take<double>(1);
  b.t_dev = cv.take<long long>(1);
  b.t_zero = cv.take<long long>(1);
  b.tau = cv.take<double>(1);
  b.flag = cv.take<int>(2);  // [0] numeric failure (sticky), [1] input check
  b.obs_w = cv.take<Real>(nn);
  b.obs_d = cv.take<Real>(nn);
  b.logk = cv.take<Real>(nn);
  b.lk_m = cv.take<Real>(nn);
  b.lk_v = cv.take<Real>(nn);
  b.t_k = cv.take<long long>(1);
  return (cv.off + 255) & ~size_t(255);
}

static crv_status validate_config(const crv_config* c) {
  if (!c) return fail(CRV_EINVAL, "config is NULL");
  if (c->dim != 2 && c->dim != 3) return fail(CRV_EINVAL, "dim must be 2 or 3");
  if (c->n_elem < 4 || c->n_elem > (c->dim == 2 ? 1024 : 256))
    return fail(CRV_EINVAL, "n_elem must be in [4, 1024] (2D) or [4, 256] (3D)");
  if (c->degree < 1 || c->degree > 3) return fail(CRV_EINVAL, "degree must be 1, 2 or 3");
  if (!(c->width == 16 || c->width == 32 || c->width == 64 || c->width == 128))
    return fail(CRV_EINVAL, "width must be 16, 32, 64 or 128");
  if (c->hidden < 1 || c->hidden > 8) return fail(CRV_EINVAL, "hidden must be in [1, 8]");
  if (c->precision < CRV_PREC_FP32 || c->precision > CRV_PREC_BF16X3F)
    return fail(CRV_EINVAL, "unknown precision");
  if ((c->precision == CRV_PREC_BF16 || c->precision == CRV_PREC_BF16X3 ||
       c->precision == CRV_PREC_BF16X3F) &&
      !mlp_mfma_supported(c->dim, c->width, c->hidden, net_mode(*c)))
    return fail(CRV_EINVAL, "bf16 network paths need width 32 or 64 (bf16 and the mixed form also "
                            "128) and 3 or 4 hidden layers (4 in 3D)");
  if (!(c->mu_w > 0) || !(c->mu_g > 0)) return fail(CRV_EINVAL, "viscosities must be > 0");
  if (!(c->relperm_exp >= 1)) return fail(CRV_EINVAL, "relperm_exp must be >= 1");
  if (!(c->lr > 0) || !(c->beta1 >= 0 && c->beta1 < 1) || !(c->beta2 >= 0 && c->beta2 < 1) ||
      !(c->eps >= 0))
    return fail(CRV_EINVAL, "bad Adam parameters");
  if (c->adam_iters < 0 || c->substeps < 1) return fail(CRV_EINVAL, "bad iteration counts");
  if (!(c->well_radius > 0)) return fail(CRV_EINVAL, "well_radius must be > 0");
  if (!(c->gravity >= 0 && std::isfinite(c->gravity)) || !(c->rho_w >= 0 && std::isfinite(c->rho_w)) ||
      !(c->rho_g >= 0 && std::isfinite(c->rho_g)))
    return fail(CRV_EINVAL, "gravity and densities must be finite and >= 0");
  if (c->boundary_factor != 0 && c->boundary_factor != 1)
    return fail(CRV_EINVAL, "boundary_factor must be 0 (indicator) or 1 (distance factor)");
  return CRV_OK;
}

// ---------------------------------------------------------------------------
struct SolverBase {
  crv_config cfg;
  Geom g;
  hipStream_t st = nullptr;
  int64_t P = 0;
  bool owns_ws = false;
  void* ws = nullptr;
  bool pretrained = false;

  // ---- event timing of kernel launches ----
  bool prof = false;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  int open_k = -1;
  hipEvent_t open_ev = nullptr;
  hipEvent_t next_event() {
    if (pool_used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[pool_used++];
  }
  void tb(int k) {
    if (!prof) return;
    open_k = k;
    open_ev = next_event();
    if (open_ev) hipEventRecord(open_ev, st);
  }
  void te() {
    if (!prof || open_k < 0) return;
    hipEvent_t e = next_event();
    if (e && open_ev) {
      hipEventRecord(e, st);
      marks.push_back({open_k, {open_ev, e}});
    }
    open_k = -1;
  }
  void profile_reset() {
    marks.clear();
    pool_used = 0;
  }

  virtual ~SolverBase() {
    for (auto e : pool) (void)hipEventDestroy(e);
    if (owns_ws && ws) (void)hipFree(ws);
  }
  virtual crv_status init(const double*, const double*, const double*, int, const double*,
                          const double*) = 0;
  virtual crv_status train(int iters) = 0;
  virtual crv_status step(double dt) = 0;
  virtual crv_status fields(double*, double*, double*) = 0;
  virtual crv_status loss_grad(double*, double*, double*) = 0;
  virtual crv_status get_state(double*, double*, double*, int64_t*) = 0;
  virtual crv_status set_state(const double*, const double*, const double*, int64_t) = 0;
  virtual crv_status set_saturation(const double*) = 0;
  virtual crv_status set_log_perm(const double*) = 0;
  virtual crv_status loss_grad_device(double*, float*, float*) = 0;
  virtual crv_status set_params_device(const float*, const float*) = 0;
  virtual crv_status set_observations(const double*, const double*) = 0;
  virtual crv_status invert(int iters, double lr_logk) = 0;
  virtual crv_status get_log_perm(double*) = 0;
  virtual crv_status loss_history(double*, int, int*) = 0;
  virtual crv_status gram_solve_host(const double*, double*) = 0;
  virtual crv_status mass_solve_host(const double*, double*) = 0;
  virtual crv_status project_host(double*) = 0;
  virtual crv_status substeps(double tau, int n) = 0;
  virtual crv_status sync() = 0;
  virtual crv_status pressure_galerkin(int max_iters, double rtol, int precond, double* p,
                                       int* iters, double* relres) = 0;
  virtual crv_status step_galerkin(double dt, int max_iters, double rtol, int precond,
                                   int* iters, double* relres) = 0;
  // scenario batching (2D float32 matrix-core contexts of one configuration)
  virtual bool batchable() const { return false; }
  virtual int64_t batch_tag() const { return 0; }
  // part: 0 = every scenario keeps its own backward grid (bitwise single
  // steps); p >= 1 = the batch's backward shares 1/p of the device's blocks
  virtual crv_status step_batched(SolverBase* const* all, const double* dts, int n, int64_t zb,
                                  int part) {
    (void)all, (void)dts, (void)n, (void)zb, (void)part;
    return fail(CRV_EINVAL, "this context cannot run a batched step");
  }
};

// the fields of two configurations are all equal
static bool same_config(const crv_config& a, const crv_config& b) {
  return a.dim == b.dim && a.n_elem == b.n_elem && a.degree == b.degree && a.width == b.width &&
         a.hidden == b.hidden && a.precision == b.precision && a.mu_w == b.mu_w &&
         a.mu_g == b.mu_g && a.relperm_exp == b.relperm_exp && a.lr == b.lr &&
         a.beta1 == b.beta1 && a.beta2 == b.beta2 && a.eps == b.eps &&
         a.adam_iters == b.adam_iters && a.substeps == b.substeps &&
         a.well_radius == b.well_radius && a.gravity == b.gravity && a.rho_w == b.rho_w &&
         a.rho_g == b.rho_g && a.boundary_factor == b.boundary_factor;
}

template <typename Real>
struct Solver : SolverBase {
  Buffers<Real> b;
  MlpShape ms;
  size_t nn = 0, nc = 0;
  bool mfma = false;
  int mode = NET_F32;
  int bwd_blocks = 0;
  // the scenario batch of the launches being enqueued ({1, 0}: this context)
  Batch bz{};

  // -------- host <-> device helpers --------
  crv_status upload(Real* dst, const double* src, size_t n) {
    std::vector<Real> tmp(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = Real(src[i]);
    CRV_HIP(hipMemcpyAsync(dst, tmp.data(), n * sizeof(Real), hipMemcpyHostToDevice, st));
    CRV_HIP(hipStreamSynchronize(st));
    return CRV_OK;
  }
  template <typename T>
  crv_status upload_raw(T* dst, const std::vector<T>& src) {
    CRV_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
    CRV_HIP(hipStreamSynchronize(st));
    return CRV_OK;
  }
  crv_status download(double* dst, const Real* src, size_t n) {
    std::vector<Real> tmp(n);
    CRV_HIP(hipMemcpyAsync(tmp.data(), src, n * sizeof(Real), hipMemcpyDeviceToHost, st));
    CRV_HIP(hipStreamSynchronize(st));
    for (size_t i = 0; i < n; ++i) dst[i] = double(tmp[i]);
    return CRV_OK;
  }
  crv_status check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CRV_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return CRV_OK;
  }
  crv_status sync() override { return sync_and_check(); }

  crv_status sync_and_check() {
    CRV_HIP(hipStreamSynchronize(st));
    int flag = 0;
    CRV_HIP(hipMemcpy(&flag, b.flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) return fail(CRV_ENUMERIC, "non-finite saturation or loss");
    return CRV_OK;
  }

  crv_status init(const double* log_perm, const double* poro, const double* wells, int n_wells,
                  const double* s0, const double* theta0) override {
    nn = size_t(ipow(g.n, g.dim));
    nc = size_t(ipow(g.nb, g.dim));
    ms = MlpShape{cfg.dim, cfg.width, cfg.hidden, P};
    mfma = uses_mfma(cfg);
    mode = net_mode(cfg);
    if (mfma) {
      int dev = 0, cus = kMaxCUs;
      CRV_HIP(hipGetDevice(&dev));
      CRV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      bwd_blocks = std::min(b.bwd_rows, mlp_bwd_mfma_blocks(g, cfg.width, cfg.hidden, mode,
                                                            std::min(cus, kMaxCUs), true));
    }
    for (size_t i = 0; i < nn; ++i) {
      if (!std::isfinite(log_perm[i])) return fail(CRV_EINVAL, "log_perm has non-finite entries");
      if (!(poro[i] > 0) || !std::isfinite(poro[i])) return fail(CRV_EINVAL, "porosity must be > 0");
    }
    if (n_wells < 0 || (n_wells > 0 && !wells)) return fail(CRV_EINVAL, "bad well list");
    for (int w = 0; w < n_wells; ++w)
      for (int k = 0; k < 3; ++k)
        if (!std::isfinite(wells[3 * w + k])) return fail(CRV_EINVAL, "well entries must be finite");
    if (s0)
      for (size_t i = 0; i < nc; ++i)
        if (!std::isfinite(s0[i])) return fail(CRV_EINVAL, "s0 has non-finite entries");
    for (int64_t i = 0; i < P; ++i)
      if (!std::isfinite(theta0[i])) return fail(CRV_EINVAL, "theta0 has non-finite entries");

    // zero the whole workspace (padding of interior arrays must stay finite)
    {
      Carve dry(nullptr);
      Buffers<Real> tmpb;
      const size_t bytes = carve<Real>(dry, cfg, tmpb);
      CRV_HIP(hipMemsetAsync(ws, 0, bytes, st));
    }
    std::string err;
    std::vector<double> qi, qp;
    if (!well_sources(wells, n_wells, g.ne, g.dim, cfg.well_radius, qi, qp, err))
      return fail(CRV_EINVAL, err);
    const double h = 1.0 / g.ne;
    const double hd = std::pow(h, g.dim);
    std::vector<double> perm(nn), hq(nn);
    for (size_t i = 0; i < nn; ++i) {
      perm[i] = std::exp(log_perm[i]);
      hq[i] = hd * (qi[i] + qp[i]);
    }
    crv_status s;
    if ((s = upload(b.perm, perm.data(), nn))) return s;
    if ((s = upload(b.logk, log_perm, nn))) return s;
    if ((s = upload(b.poro, poro, nn))) return s;
    if ((s = upload(b.qi, qi.data(), nn))) return s;
    if ((s = upload(b.qp, qp.data(), nn))) return s;
    if ((s = upload(b.hq, hq.data(), nn))) return s;
    if (s0 && (s = upload(b.s, s0, nc))) return s;
    if ((s = upload(b.theta, theta0, size_t(P)))) return s;

    // discretisation tables (float64 on the host)
    std::vector<int> kf, pf;
    std::vector<double> kv, pv, gbv, gdbv, gxi, gw;
    knot_table(g.ne, g.r, kf, kv);
    projection_table(g.ne, g.r, pf, pv);
    gauss_tables(g.ne, g.r, gbv, gdbv, gxi, gw);
    if ((s = upload_raw(b.knot_first, kf))) return s;
    if ((s = upload(b.knot_val, kv.data(), kv.size()))) return s;
    if ((s = upload(b.proj_val, pv.data(), pv.size()))) return s;
    if ((s = upload(b.gb, gbv.data(), gbv.size()))) return s;
    if ((s = upload(b.gdb, gdbv.data(), gdbv.size()))) return s;
    if ((s = upload(b.gxi, gxi.data(), gxi.size()))) return s;
    if ((s = upload(b.gw, gw.data(), gw.size()))) return s;
    std::vector<double> dst, lam;
    dst_table(g.m, g.mp, dst, lam);
    if ((s = upload(b.dst, dst.data(), dst.size()))) return s;
    {
      const std::vector<double> pk = pack_gemm_a(dst, g.mp, g.mp);
      if ((s = upload(b.dst_pk, pk.data(), pk.size()))) return s;
    }
    // shift of each line: lambda_j (2D), lambda_j + lambda_k (3D, padded
    // modes get a harmless positive shift; their lines hold zeros)
    std::vector<double> shifts(size_t(gram_lines(g)));
    if (g.dim == 2) {
      for (int j = 0; j < g.m; ++j) shifts[j] = lam[j];
    } else {
      for (int k = 0; k < g.m; ++k)
        for (int j = 0; j < g.mp; ++j) shifts[size_t(k) * g.mp + j] = lam[k] + (j < g.m ? lam[j] : 2.0);
    }
    if ((s = upload_raw(b.shifts, shifts))) return s;
    std::vector<double> band = mass_band(g.ne, g.r);
    if ((s = upload_raw(b.band, band))) return s;

    // float64 factorisations on the device (eq. 14 mass band, eq. 28 Gram lines)
    launch_factor_band<Real>(b.band, g.nb, g.r, b.band_work, b.m_lt, b.m_invd, b.status, st);
    // G = L5 in 2D, h L7 in 3D
    launch_factor_shifted<Real>(b.shifts, int(gram_lines(g)), g.m, g.mp, g.dim == 3 ? h : 1.0,
                                b.g_lt, b.g_invd, st);
    if ((s = check_launch())) return s;
    refresh();
    pack();
    if ((s = check_launch())) return s;
    CRV_HIP(hipStreamSynchronize(st));
    int status = 0;
    CRV_HIP(hipMemcpy(&status, b.status, sizeof(int), hipMemcpyDeviceToHost));
    if (status) return fail(CRV_ENUMERIC, "mass matrix factorisation failed");
    return CRV_OK;
  }

  // alpha (and with gravity the buoyancy flux and the pressure right-hand
  // side, which then depend on S) from the current saturation
  bool gravity() const { return cfg.gravity != 0.0; }
  void refresh() {
    tb(CRV_K_REFRESH);
    launch_refresh<Real>(g, b.s, b.knot_first, b.knot_val, b.perm, cfg.mu_w, cfg.mu_g,
                         cfg.relperm_exp, cfg.rho_w, cfg.rho_g, b.s_nodal, b.alpha,
                         gravity() ? b.gflux : nullptr, st, bz);
    if (gravity()) launch_gravity_rhs<Real>(g, b.gflux, b.qi, b.qp, cfg.gravity, b.hq, st, bz);
    te();
  }

  // q = G^-1 res: DST-I along y (product with the orthonormal sine basis),
  // shifted tridiagonal solves along x, inverse DST-I along y (eq. 26-28).
  // 3D: DST-I along z (one product over all (y, x) columns) and along y (one
  // product per z plane), lines along x with shift lambda_j + lambda_k.
  void gram_solve() {
    const int mp = g.mp;
    const int64_t mp2 = int64_t(mp) * mp;
    if (g.dim == 3) {
      tb(CRV_K_GRAM_DST);
      launch_gemm<Real>(mp, int(mp2), mp, b.dst, mp, b.res, int(mp2), b.qhat, int(mp2), st, b.dst_pk);
      launch_gemm_batched<Real>(mp, mp, mp, b.dst, mp, b.qhat, mp, mp2, b.rhat, mp, mp2, mp, st, b.dst_pk);
      te();
      tb(CRV_K_GRAM_LINES);
      launch_band_rows<Real>(b.rhat, b.qhat, g.m, int(gram_lines(g)), mp, 1, b.g_lt, b.g_invd, mp,
                             mp, st);
      te();
      tb(CRV_K_GRAM_DST);
      launch_gemm_batched<Real>(mp, mp, mp, b.dst, mp, b.qhat, mp, mp2, b.rhat, mp, mp2, mp, st, b.dst_pk);
      launch_gemm<Real>(mp, int(mp2), mp, b.dst, mp, b.rhat, int(mp2), b.q, int(mp2), st, b.dst_pk);
      te();
      return;
    }
    // a scenario batch is the batch of the products (the sine basis, the A
    // operand, is the same table in every scenario's workspace)
    const int64_t zs = bz.zb / int64_t(sizeof(Real));
    tb(CRV_K_GRAM_DST);
    launch_gemm_batched<Real>(mp, mp, mp, b.dst, mp, b.res, mp, zs, b.rhat, mp, zs, bz.n, st, b.dst_pk);
    te();
    tb(CRV_K_GRAM_LINES);
    launch_band_rows<Real>(b.rhat, b.qhat, g.m, g.m, mp, 1, b.g_lt, b.g_invd, mp, mp, st, bz);
    te();
    tb(CRV_K_GRAM_DST);
    launch_gemm_batched<Real>(mp, mp, mp, b.dst, mp, b.qhat, mp, zs, b.q, mp, zs, bz.n, st, b.dst_pk);
    te();
  }

  // dst = (M^x (x) M^y [(x) M^z])^-1 src (eq. 14): x-lines src -> dst, then
  // y-lines (per z plane) and z-lines in place.
  void mass_solve(const Real* src, Real* dst) {
    const int nb = g.nb;
    const int64_t nb2 = int64_t(nb) * nb;
    tb(CRV_K_MASS_ROWS);
    launch_band_rows<Real>(src, dst, nb, g.dim == 3 ? int(nb2) : nb, nb, g.r, b.m_lt, b.m_invd, 0,
                           0, st, bz);
    te();
    tb(CRV_K_MASS_COLS);
    launch_band_cols<Real>(dst, dst, nb, nb, nb, g.r, b.m_lt, b.m_invd, g.dim == 3 ? nb : 1,
                           g.dim == 3 ? nb2 : 0, st, bz);
    if (g.dim == 3)
      launch_band_cols<Real>(dst, dst, nb, int(nb2), nb2, g.r, b.m_lt, b.m_invd, 1, 0, st);
    te();
  }

  // robust loss, g_u and the loss value (slot given by hist/t)
  // weight fragments of the matrix-core kernels follow every change of theta
  void pack() {
    if constexpr (std::is_same<Real, float>::value) {
      if (mfma) launch_pack_fragments(b.theta, cfg.dim, cfg.width, cfg.hidden, mode, b.frag, st);
    }
  }

  // network forward into b.u; t_bump (nullable) marks the start of an Adam iteration
  void forward(long long* t_bump = nullptr) {
    tb(CRV_K_MLP_FWD);
    if constexpr (std::is_same<Real, float>::value) {
      if (mfma) {
        launch_mlp_forward_mfma(g, cfg.width, cfg.hidden, mode, b.theta, b.frag, b.u, t_bump, st, bz);
        te();
        return;
      }
    }
    launch_mlp_forward<Real>(g, ms, b.theta, b.u, t_bump, st);
    te();
  }

  // forward, residual, Gram solve and (unless the matrix-core backward fuses
  // it) the adjoint: b.u, b.res, b.q, b.gu and the per-block loss partials
  void loss_pass(long long* t_bump) {
    forward(t_bump);
    tb(CRV_K_RESIDUAL);
    launch_residual<Real>(g, b.u, b.alpha, b.hq, b.res, st, bz);
    te();
    gram_solve();
    if (mfma) return;
    tb(CRV_K_ADJOINT);
    adj_np = launch_adjoint<Real>(g, b.q, b.alpha, b.res, b.gu, b.loss_part, st,
                                  obs_on ? b.obs_w : nullptr, b.obs_d, b.u);
    te();
  }

  // pressure observations of the inverse problem are in use (they change
  // the captured work, so switching them on or off drops the graphs)
  bool obs_on = false;

  // partial gradient rows of the network backward; returns the row count.
  // The matrix-core backward also leaves one loss partial per block.  A
  // batch keeps each scenario's own grid (bitwise a single step), unless it
  // shares the blocks that fit on the device at once among its n scenarios
  // (about bwd_blocks / n each; / (n p) when the batch is to take 1/p of the
  // device, leaving room for other streams' batches): then all of them run
  // in one round and each writes that many times fewer partial rows, its
  // gradient sums rounding differently from a single step's (the same sums,
  // grouped otherwise).
  int share_part = 0;  // 0: own grid per scenario; p: the batch shares 1/p of the device's blocks
  int bwd_grid() const {
    if (bz.n <= 1 || share_part <= 0) return bwd_blocks;
    const int per = bz.n * share_part;
    return std::max(1, (bwd_blocks + per - 1) / per);
  }
  int adj_np = 0;
  int64_t ldp() const { return partial_pitch(P); }  // pitch of the matrix-core partial rows
  int loss_count() const { return mfma ? bwd_grid() : adj_np; }
  int backward() {
    tb(CRV_K_MLP_BWD);
    int rows = 0;
    if constexpr (std::is_same<Real, float>::value) {
      if (mfma) {
        launch_mlp_backward_mfma(g, cfg.width, cfg.hidden, mode, ldp(), b.theta, b.frag, b.q, b.alpha,
                                 b.res, b.partials, b.loss_part, bwd_grid(), st, bz,
                                 obs_on ? b.obs_w : nullptr, b.obs_d, b.u);
        rows = bwd_grid();
      }
    }
    if (!rows) rows = launch_mlp_backward<Real>(g, ms, b.theta, b.gu, b.partials, st);
    te();
    return rows;
  }

  void grad_pass() {
    const int rows = backward();
    tb(CRV_K_GRAD_REDUCE);
    launch_reduce_rows<Real>(b.partials, rows, P, mfma ? ldp() : P, b.red_scratch, b.grad, st);
    te();
  }

  // one Adam iteration: the forward advances the step counter t, the loss
  // of the iteration lands in loss_hist[(t-1) % cap]
  void iteration() {
    loss_pass(b.t_dev);
    if constexpr (std::is_same<Real, float>::value) {
      if (mfma) {
        const int rows = backward();
        tb(CRV_K_ADAM);
        launch_reduce_adam_pack(b.partials, rows, P, ldp(), b.theta, b.am, b.av, cfg.lr, cfg.beta1,
                                cfg.beta2, cfg.eps, b.t_dev, cfg.dim, cfg.width, cfg.hidden, mode,
                                b.frag, b.loss_part, loss_count(), b.loss_hist, kLossCap, st, bz);
        te();
        return;
      }
    }
    tb(CRV_K_LOSS);
    launch_loss_finalize<Real>(b.loss_part, loss_count(), b.loss_hist, kLossCap, b.t_dev, -1, st);
    te();
    grad_pass();
    tb(CRV_K_ADAM);
    launch_adam<Real>(P, b.theta, b.am, b.av, b.grad, cfg.lr, cfg.beta1, cfg.beta2, cfg.eps,
                      b.t_dev, st);
    pack();
    te();
  }

  // ---- captured work: one hipGraph per sequence, replayed on the caller's stream ----
  hipStream_t cap = nullptr;
  hipGraphExec_t g_train = nullptr, g_step = nullptr;
  bool graphs_off = std::getenv("CRV_NO_GRAPH") != nullptr;

  // ---- IGA Galerkin pressure (the paper's direct-solver path, 2D) ----
  GalerkinWork<Real> gw{};
  void* gw_mem = nullptr;
  hipGraphExec_t g_gal[2] = {nullptr, nullptr};  // a captured chunk of CG iterations per preconditioner
  crv_status galerkin_alloc() {
    if (gw_mem) return CRV_OK;
    const size_t npts = size_t(ipow(int64_t(g.ne) * (g.r + 1), 2)), ncf = size_t(g.nb) * g.nb;
    auto up = [](size_t bytes) { return (bytes + 255) & ~size_t(255); };
    const size_t nparts = size_t(galerkin_partials(g));
    gw.mg = g.nb - 2;
    gw.mgp = (gw.mg + 63) / 64 * 64;
    const size_t mp2 = size_t(gw.mgp) * gw.mgp;
    const size_t bytes = 3 * up(npts * sizeof(Real)) + 8 * up(ncf * sizeof(Real)) +
                         up(8 * sizeof(double)) + 2 * up(2 * nparts * sizeof(double)) +
                         5 * up(mp2 * sizeof(Real)) + up(2 * size_t(gw.mgp) * sizeof(Real));
    CRV_HIP(hipMalloc(&gw_mem, bytes));
    Carve cv(gw_mem);
    gw.c = cv.take<Real>(npts);
    gw.f0 = cv.take<Real>(npts);
    gw.fy = cv.take<Real>(npts);
    gw.f = cv.take<Real>(ncf);
    gw.dg = cv.take<Real>(ncf);
    gw.r = cv.take<Real>(ncf);
    gw.z = cv.take<Real>(ncf);
    gw.p = cv.take<Real>(ncf);
    gw.p2 = cv.take<Real>(ncf);
    gw.ap = cv.take<Real>(ncf);
    gw.sc = cv.take<double>(8);
    gw.part = cv.take<double>(2 * nparts);
    gw.part2 = cv.take<double>(2 * nparts);
    gw.ksc = cv.take<Real>(ncf);
    gw.kt0 = cv.take<Real>(mp2);
    gw.kt1 = cv.take<Real>(mp2);
    gw.kt2 = cv.take<Real>(mp2);
    gw.kdst = cv.take<Real>(mp2);
    gw.kdst_pk = cv.take<Real>(mp2);
    gw.ksym = cv.take<Real>(2 * size_t(gw.mgp));
    std::vector<double> dst, lam, sym;
    dst_table(gw.mg, gw.mgp, dst, lam);
    bspline_symbols(g.r, gw.mg, gw.mgp, sym);
    crv_status s;
    if ((s = upload(gw.kdst, dst.data(), dst.size()))) return s;
    {
      const std::vector<double> pk = pack_gemm_a(dst, gw.mgp, gw.mgp);
      if ((s = upload(gw.kdst_pk, pk.data(), pk.size()))) return s;
    }
    if ((s = upload(gw.ksym, sym.data(), sym.size()))) return s;
    CRV_HIP(hipStreamSynchronize(st));
    return CRV_OK;
  }
  GalerkinArgs<Real> galerkin_args(int precond) {
    return GalerkinArgs<Real>{b.s, b.perm, b.qi, b.qp, b.gb, b.gdb, b.gxi, b.gw,
                              cfg.mu_w, cfg.mu_g, cfg.relperm_exp, cfg.rho_w, cfg.rho_g,
                              cfg.gravity, b.p, gw, precond};
  }
  // S P = F for the current saturation into b.p by preconditioned CG from
  // P = 0, until |r| <= rtol |F| (tested after every iteration on the device)
  // or max_iters.  Iterations run in chunks of 24 (a captured graph) and
  // alternate the slot of r.z, so every chunk but the last (which may be
  // shorter) has an even length
  crv_status pressure_galerkin(int max_iters, double rtol, int precond, double* p_out,
                               int* iters_out, double* relres_out) override {
    if (g.dim != 2) return fail(CRV_EINVAL, "the Galerkin pressure path is built for 2D");
    if (max_iters < 0 || !(rtol >= 0) || !std::isfinite(rtol)) return fail(CRV_EINVAL, "bad max_iters or rtol");
    if (precond != CRV_PRECOND_JACOBI && precond != CRV_PRECOND_KRON)
      return fail(CRV_EINVAL, "precond must be CRV_PRECOND_JACOBI or CRV_PRECOND_KRON");
    crv_status s = galerkin_alloc();
    if (s) return s;
    const GalerkinArgs<Real> a = galerkin_args(precond);
    // slots 5-7 (stop flag, threshold, iteration count): no stop before the
    // threshold is known
    double tail[3] = {0.0, -1.0, 0.0};
    auto write_tail = [&]() -> crv_status {
      CRV_HIP(hipMemcpyAsync(gw.sc + 5, tail, sizeof(tail), hipMemcpyHostToDevice, st));
      CRV_HIP(hipStreamSynchronize(st));
      return CRV_OK;
    };
    if ((s = write_tail())) return s;
    launch_galerkin_setup<Real>(g, a, st);
    if ((s = check_launch())) return s;
    double sc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    auto read_sc = [&]() -> crv_status {
      CRV_HIP(hipMemcpyAsync(sc, gw.sc, sizeof(sc), hipMemcpyDeviceToHost, st));
      CRV_HIP(hipStreamSynchronize(st));
      return CRV_OK;
    };
    if ((s = read_sc())) return s;
    const double ff = sc[4];
    double rel = ff > 0 ? 1.0 : 0.0;
    // the iterations stop themselves on the device once r.r <= rtol^2 F.F, so
    // a chunk may end early and the count comes from the device.  Slots 1-7:
    // the r.z before the first iteration (0: no previous direction), unused,
    // r.r = F.F (r = F), F.F, flag, threshold, count
    {
      const double head[7] = {0.0, 0.0, ff, ff, 0.0, rtol * rtol * ff, 0.0};
      CRV_HIP(hipMemcpyAsync(gw.sc + 1, head, sizeof(head), hipMemcpyHostToDevice, st));
      CRV_HIP(hipStreamSynchronize(st));
    }
    int done = 0;
    const int chunk = 24;  // even: each chunk starts with rz in slot 0
    hipGraphExec_t& graph = g_gal[precond];
    if (use_graphs() && !graph && ff > 0 && max_iters >= chunk) {
      s = capture(&graph, [&] { launch_galerkin_iters<Real>(g, a, chunk, st); });
      if (s) return s;
    }
    bool stopped = false;
    while (ff > 0 && done < max_iters && rel > rtol && !stopped) {
      const int k = std::min(chunk, max_iters - done);
      if (graph && use_graphs() && k == chunk) CRV_HIP(hipGraphLaunch(graph, st));
      else launch_galerkin_iters<Real>(g, a, k, st);
      if ((s = check_launch())) return s;
      if ((s = read_sc())) return s;
      done += k;
      stopped = sc[5] != 0.0;
      if (!std::isfinite(sc[3])) return fail(CRV_ENUMERIC, "Galerkin solve produced a non-finite residual");
    }
    if (ff > 0) {
      launch_galerkin_finish<Real>(gw, st);
      if ((s = check_launch())) return s;
      if ((s = read_sc())) return s;
      rel = std::sqrt(std::max(sc[3], 0.0) / ff);
      if (!std::isfinite(rel)) return fail(CRV_ENUMERIC, "Galerkin solve produced a non-finite residual");
    }
    done = int(sc[7]);
    if (iters_out) *iters_out = done;
    if (relres_out) *relres_out = rel;
    if (p_out && (s = download(p_out, b.p, nc))) return s;
    return CRV_OK;
  }
  // the direct-solver algorithm's pass: substeps with the current pressure
  // coefficients, refresh, and the Galerkin pressure of the new saturation
  crv_status step_galerkin(double dt, int max_iters, double rtol, int precond, int* iters,
                           double* relres) override {
    if (g.dim != 2) return fail(CRV_EINVAL, "the Galerkin pressure path is built for 2D");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(CRV_EINVAL, "dt must be > 0");
    crv_status s = set_tau(dt / cfg.substeps);
    if (s) return s;
    for (int k = 0; k < cfg.substeps; ++k) substep();
    launch_check_finite<Real>(b.s, nc, b.flag, st);
    refresh();
    if ((s = check_launch())) return s;
    if ((s = sync_and_check())) return s;
    return pressure_galerkin(max_iters, rtol, precond, nullptr, iters, relres);
  }

  ~Solver() override {
    for (BatchGraph& bg : g_batch) (void)hipGraphExecDestroy(bg.exec);
    for (hipEvent_t e : join_ev) (void)hipEventDestroy(e);
    for (hipGraphExec_t& e : g_gal)
      if (e) (void)hipGraphExecDestroy(e);
    if (gw_mem) (void)hipFree(gw_mem);
    if (g_train) (void)hipGraphExecDestroy(g_train);
    if (g_step) (void)hipGraphExecDestroy(g_step);
    if (cap) (void)hipStreamDestroy(cap);
  }

  template <typename F>
  crv_status capture(hipGraphExec_t* out, F&& body) {
    if (!cap) CRV_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t user = st;
    st = cap;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) body();
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    st = user;
    if (e != hipSuccess) return fail(CRV_EHIP, std::string("begin capture: ") + hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(CRV_EHIP, std::string("end capture: ") + hipGetErrorString(e2));
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(CRV_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
    return CRV_OK;
  }

  bool use_graphs() const { return !prof && !graphs_off; }

  crv_status train(int iters) override {
    const int chunk = std::max(1, cfg.adam_iters);
    int done = 0;
    if (use_graphs() && iters >= chunk) {
      if (!g_train) {
        crv_status s = capture(&g_train, [&] {
          for (int i = 0; i < chunk; ++i) iteration();
        });
        if (s) return s;
      }
      for (; done + chunk <= iters; done += chunk) CRV_HIP(hipGraphLaunch(g_train, st));
    }
    for (; done < iters; ++done) iteration();
    crv_status s = check_launch();
    if (s) return s;
    pretrained = true;
    return CRV_OK;
  }

  // algorithm step 4: p = M^-1 int I_h(u) B
  void project_into_p() {
    forward();
    tb(CRV_K_PROJECT);
    launch_project<Real>(g, b.u, b.proj_val, b.bvec, st, bz);
    te();
    mass_solve(b.bvec, b.p);
  }

  // algorithm step 5 (tau from b.tau): S <- M^-1 b(S, p)
  void substep() {
    tb(CRV_K_ADS_ASSEMBLE);
    launch_ads_assemble<Real>(g, b.s, b.p, b.perm, b.poro, b.qi, b.qp, b.gb, b.gdb, b.gxi, b.gw,
                              b.tau, cfg.mu_w, cfg.mu_g, cfg.relperm_exp, cfg.rho_g * cfg.gravity,
                              b.bvec, st, bz);
    te();
    mass_solve(b.bvec, b.s);
  }

  void step_body() {
    project_into_p();
    for (int k = 0; k < cfg.substeps; ++k) substep();
    launch_check_finite<Real>(b.s, nc, b.flag, st, bz);
    refresh();
    for (int i = 0; i < cfg.adam_iters; ++i) iteration();
  }

  // tau into device memory by a one-thread kernel: stream-ordered before the
  // step that reads it, and the host does not wait
  crv_status set_tau(double tau) {
    launch_set_f64(b.tau, tau, st);
    return check_launch();
  }

  crv_status step(double dt) override {
    if (!(dt > 0) || !std::isfinite(dt)) return fail(CRV_EINVAL, "dt must be > 0");
    crv_status s = set_tau(dt / cfg.substeps);
    if (s) return s;
    if (use_graphs()) {
      if (!g_step) {
        s = capture(&g_step, [&] { step_body(); });
        if (s) return s;
      }
      CRV_HIP(hipGraphLaunch(g_step, st));
    } else {
      step_body();
    }
    return check_launch();
  }

  // ---- batched coupled step ----
  // Scenarios of this context's configuration whose workspaces lie zb bytes
  // apart, starting with this one, advance together: every kernel of the step
  // runs once for all of them (blockIdx.z selects the scenario), replayed
  // from a graph captured per (count, stride, sharing) on this context's
  // stream.  Without sharing every kernel reduces in an order that does not
  // depend on the batch, so each scenario's result is bitwise the one of its
  // own crv_step; with sharing the backward's grouping differs (above).
  struct BatchGraph {
    int n;
    int64_t zb;
    int part;
    hipGraphExec_t exec;
  };
  std::vector<BatchGraph> g_batch;
  std::vector<hipEvent_t> join_ev;

  bool batchable() const override {
    return std::is_same<Real, float>::value && mfma && g.dim == 2;
  }
  int64_t batch_tag() const override { return bwd_blocks; }

  hipEvent_t join_event(size_t k) {
    while (join_ev.size() <= k) {
      hipEvent_t e = nullptr;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
      join_ev.push_back(e);
    }
    return join_ev[k];
  }

  crv_status step_batched(SolverBase* const* all, const double* dts, int n, int64_t zb,
                          int part) override {
    // order after the work already queued on the other scenarios' streams
    size_t ev = 0;
    for (int k = 1; k < n; ++k) {
      if (all[k]->st == st) continue;
      hipEvent_t e = join_event(ev++);
      if (!e) return fail(CRV_EHIP, "hipEventCreate failed");
      CRV_HIP(hipEventRecord(e, all[k]->st));
      CRV_HIP(hipStreamWaitEvent(st, e, 0));
    }
    std::vector<double> taus(static_cast<size_t>(n));
    for (int k = 0; k < n; ++k) taus[k] = dts[k] / cfg.substeps;
    launch_set_f64_batch(b.tau, zb, taus.data(), n, st);
    crv_status s = check_launch();
    if (s) return s;
    const Batch one = bz;
    if (use_graphs()) {
      hipGraphExec_t exec = nullptr;
      for (const BatchGraph& bg : g_batch)
        if (bg.n == n && bg.zb == zb && bg.part == part) exec = bg.exec;
      if (!exec) {
        bz = Batch{n, zb};
        share_part = part;
        s = capture(&exec, [&] { step_body(); });
        bz = one;
        share_part = 0;
        if (s) return s;
        g_batch.push_back(BatchGraph{n, zb, part, exec});
      }
      CRV_HIP(hipGraphLaunch(exec, st));
    } else {
      bz = Batch{n, zb};
      share_part = part;
      step_body();
      bz = one;
      share_part = 0;
    }
    if ((s = check_launch())) return s;
    // and the other streams' later work after the batch
    hipEvent_t done = join_event(ev);
    if (!done) return fail(CRV_EHIP, "hipEventCreate failed");
    bool recorded = false;
    for (int k = 1; k < n; ++k) {
      if (all[k]->st == st) continue;
      if (!recorded) {
        CRV_HIP(hipEventRecord(done, st));
        recorded = true;
      }
      CRV_HIP(hipStreamWaitEvent(all[k]->st, done, 0));
    }
    return CRV_OK;
  }

  crv_status substeps(double tau, int n) override {
    if (!(tau > 0) || !std::isfinite(tau) || n < 0) return fail(CRV_EINVAL, "bad tau or count");
    crv_status s = set_tau(tau);
    if (s) return s;
    project_into_p();
    for (int k = 0; k < n; ++k) substep();
    launch_check_finite<Real>(b.s, nc, b.flag, st);
    refresh();
    s = check_launch();
    if (s) return s;
    return sync_and_check();
  }

  crv_status fields(double* p_nodal, double* s_coefs, double* s_nodal) override {
    forward();
    crv_status s = check_launch();
    if (s) return s;
    if ((s = sync_and_check())) return s;
    if (p_nodal && (s = download(p_nodal, b.u, nn))) return s;
    if (s_coefs && (s = download(s_coefs, b.s, nc))) return s;
    if (s_nodal && (s = download(s_nodal, b.s_nodal, nn))) return s;
    return CRV_OK;
  }

  crv_status loss_grad(double* loss, double* dtheta, double* dlogperm) override {
    loss_pass(nullptr);
    grad_pass();
    launch_loss_finalize<Real>(b.loss_part, loss_count(), b.loss_scalar, 1, b.t_zero, 0, st);
    if (dlogperm)
      launch_grad_logperm<Real>(g, b.u, b.q, b.alpha, gravity() ? b.gflux : nullptr, cfg.gravity,
                                b.tmp_nodal, st);
    crv_status s = check_launch();
    if (s) return s;
    CRV_HIP(hipStreamSynchronize(st));
    if (loss) CRV_HIP(hipMemcpy(loss, b.loss_scalar, sizeof(double), hipMemcpyDeviceToHost));
    if (dtheta && (s = download(dtheta, b.grad, size_t(P)))) return s;
    if (dlogperm && (s = download(dlogperm, b.tmp_nodal, nn))) return s;
    return CRV_OK;
  }

  crv_status get_state(double* th, double* m, double* v, int64_t* t) override {
    crv_status s;
    CRV_HIP(hipStreamSynchronize(st));
    if (th && (s = download(th, b.theta, size_t(P)))) return s;
    if (m && (s = download(m, b.am, size_t(P)))) return s;
    if (v && (s = download(v, b.av, size_t(P)))) return s;
    if (t) {
      long long tt = 0;
      CRV_HIP(hipMemcpy(&tt, b.t_dev, sizeof(tt), hipMemcpyDeviceToHost));
      *t = tt;
    }
    return CRV_OK;
  }

  crv_status set_state(const double* th, const double* m, const double* v, int64_t t) override {
    if (t < -1) return fail(CRV_EINVAL, "t must be >= 0 (or -1 to keep it)");
    crv_status s;
    CRV_HIP(hipStreamSynchronize(st));
    if (th && (s = upload(b.theta, th, size_t(P)))) return s;
    if (m && (s = upload(b.am, m, size_t(P)))) return s;
    if (v && (s = upload(b.av, v, size_t(P)))) return s;
    pack();
    if ((s = check_launch())) return s;
    if (t >= 0) {
      long long tt = t;
      CRV_HIP(hipMemcpy(b.t_dev, &tt, sizeof(tt), hipMemcpyHostToDevice));
      pretrained = true;
    }
    return CRV_OK;
  }

  crv_status set_log_perm(const double* lk) override {
    std::vector<double> perm(nn);
    for (size_t i = 0; i < nn; ++i) {
      if (!std::isfinite(lk[i])) return fail(CRV_EINVAL, "log_perm has non-finite entries");
      perm[i] = std::exp(lk[i]);
    }
    CRV_HIP(hipStreamSynchronize(st));
    crv_status s = upload(b.perm, perm.data(), nn);
    if (s) return s;
    if ((s = upload(b.logk, lk, nn))) return s;
    refresh();
    return check_launch();
  }

  // ---- differentiation form on device arrays (float32 contexts) ----
  // p must be device memory: a host pointer handed to a kernel or a
  // device-to-device copy would fault instead of failing
  crv_status check_device_ptr(const void* p, const char* what) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
      (void)hipGetLastError();  // the query's failure is not a launch error
      return fail(CRV_EINVAL, std::string(what) + " is not device memory");
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
      return fail(CRV_EINVAL, std::string(what) + " is not device memory");
    return CRV_OK;
  }

  crv_status loss_grad_device(double* d_loss, float* d_dtheta, float* d_dlogperm) override {
    if constexpr (!std::is_same<Real, float>::value) {
      return fail(CRV_EINVAL, "device-array differentiation needs a float32 context");
    } else {
      crv_status s;
      if (d_loss && (s = check_device_ptr(d_loss, "loss"))) return s;
      if (d_dtheta && (s = check_device_ptr(d_dtheta, "dtheta"))) return s;
      if (d_dlogperm && (s = check_device_ptr(d_dlogperm, "dlogperm"))) return s;
      loss_pass(nullptr);
      grad_pass();
      if (d_loss) {
        launch_loss_finalize<Real>(b.loss_part, loss_count(), b.loss_scalar, 1, b.t_zero, 0, st);
        CRV_HIP(hipMemcpyAsync(d_loss, b.loss_scalar, sizeof(double), hipMemcpyDeviceToDevice, st));
      }
      if (d_dtheta)
        CRV_HIP(hipMemcpyAsync(d_dtheta, b.grad, size_t(P) * sizeof(float), hipMemcpyDeviceToDevice,
                               st));
      if (d_dlogperm) {
        launch_grad_logperm<Real>(g, b.u, b.q, b.alpha, gravity() ? b.gflux : nullptr, cfg.gravity,
                                  b.tmp_nodal, st);
        CRV_HIP(hipMemcpyAsync(d_dlogperm, b.tmp_nodal, nn * sizeof(float),
                               hipMemcpyDeviceToDevice, st));
      }
      return check_launch();
    }
  }

  crv_status set_params_device(const float* d_theta, const float* d_logperm) override {
    if constexpr (!std::is_same<Real, float>::value) {
      return fail(CRV_EINVAL, "device-array parameters need a float32 context");
    } else {
      crv_status s;
      if (d_theta && (s = check_device_ptr(d_theta, "theta"))) return s;
      if (d_logperm && (s = check_device_ptr(d_logperm, "log_perm"))) return s;
      if (d_logperm) {
        // reject non-finite log K before anything changes (one wait)
        CRV_HIP(hipMemsetAsync(b.flag + 1, 0, sizeof(int), st));
        launch_check_finite<float>(d_logperm, nn, b.flag + 1, st);
        if ((s = check_launch())) return s;
        int bad = 0;
        CRV_HIP(hipMemcpyAsync(&bad, b.flag + 1, sizeof(int), hipMemcpyDeviceToHost, st));
        CRV_HIP(hipStreamSynchronize(st));
        if (bad) return fail(CRV_EINVAL, "log_perm has non-finite entries");
      }
      if (d_theta) {
        CRV_HIP(hipMemcpyAsync(b.theta, d_theta, size_t(P) * sizeof(float),
                               hipMemcpyDeviceToDevice, st));
        pack();
      }
      if (d_logperm) {
        launch_set_logk(int64_t(nn), d_logperm, b.logk, b.perm, st);
        refresh();
      }
      return check_launch();
    }
  }

  // ---- inverse problem ----
  void drop_graphs() {
    if (g_train) (void)hipGraphExecDestroy(g_train);
    if (g_step) (void)hipGraphExecDestroy(g_step);
    g_train = g_step = nullptr;
    for (BatchGraph& bg : g_batch) (void)hipGraphExecDestroy(bg.exec);
    g_batch.clear();
  }

  crv_status set_observations(const double* data, const double* weights) override {
    const bool on = data != nullptr;
    if (on) {
      for (size_t i = 0; i < nn; ++i)
        if (!std::isfinite(data[i]) || !std::isfinite(weights[i]) || weights[i] < 0)
          return fail(CRV_EINVAL, "observations must be finite with weights >= 0");
      crv_status s = upload(b.obs_d, data, nn);
      if (s) return s;
      if ((s = upload(b.obs_w, weights, nn))) return s;
    }
    if (on != obs_on) {
      CRV_HIP(hipStreamSynchronize(st));
      drop_graphs();
    }
    obs_on = on;
    return CRV_OK;
  }

  // one joint iteration: the objective's gradients in theta and log K at the
  // current (theta, log K), Adam on theta, Adam on log K (its own moments and
  // count), K and alpha from the new log K
  void invert_iteration(double lr_logk) {
    loss_pass(b.t_dev);
    if constexpr (std::is_same<Real, float>::value) {
      if (mfma) {
        const int rows = backward();
        launch_grad_logperm<Real>(g, b.u, b.q, b.alpha, gravity() ? b.gflux : nullptr,
                                  cfg.gravity, b.tmp_nodal, st);
        launch_reduce_adam_pack(b.partials, rows, P, ldp(), b.theta, b.am, b.av, cfg.lr, cfg.beta1,
                                cfg.beta2, cfg.eps, b.t_dev, cfg.dim, cfg.width, cfg.hidden, mode,
                                b.frag, b.loss_part, loss_count(), b.loss_hist, kLossCap, st);
        invert_logk(lr_logk);
        return;
      }
    }
    launch_loss_finalize<Real>(b.loss_part, loss_count(), b.loss_hist, kLossCap, b.t_dev, -1, st);
    grad_pass();
    launch_grad_logperm<Real>(g, b.u, b.q, b.alpha, gravity() ? b.gflux : nullptr, cfg.gravity,
                              b.tmp_nodal, st);
    launch_adam<Real>(P, b.theta, b.am, b.av, b.grad, cfg.lr, cfg.beta1, cfg.beta2, cfg.eps,
                      b.t_dev, st);
    pack();
    invert_logk(lr_logk);
  }
  void invert_logk(double lr_logk) {
    launch_bump(b.t_k, st);
    launch_adam_logk<Real>(int64_t(nn), b.logk, b.lk_m, b.lk_v, b.tmp_nodal, b.perm, lr_logk,
                           cfg.beta1, cfg.beta2, cfg.eps, b.t_k, st);
    refresh();
  }
  crv_status invert(int iters, double lr_logk) override {
    if (iters < 0 || !(lr_logk >= 0) || !std::isfinite(lr_logk))
      return fail(CRV_EINVAL, "iters must be >= 0 and lr_logk finite and >= 0");
    for (int i = 0; i < iters; ++i) invert_iteration(lr_logk);
    crv_status s = check_launch();
    if (s) return s;
    return sync_and_check();
  }
  crv_status get_log_perm(double* out) override { return download(out, b.logk, nn); }

  crv_status set_saturation(const double* sc) override {
    for (size_t i = 0; i < nc; ++i)
      if (!std::isfinite(sc[i])) return fail(CRV_EINVAL, "saturation has non-finite entries");
    crv_status s = upload(b.s, sc, nc);
    if (s) return s;
    refresh();
    return check_launch();
  }

  crv_status loss_history(double* out, int cap, int* n) override {
    CRV_HIP(hipStreamSynchronize(st));
    long long t = 0;
    CRV_HIP(hipMemcpy(&t, b.t_dev, sizeof(t), hipMemcpyDeviceToHost));
    std::vector<double> h(kLossCap);
    CRV_HIP(hipMemcpy(h.data(), b.loss_hist, kLossCap * sizeof(double), hipMemcpyDeviceToHost));
    long long avail = std::min<long long>(t, kLossCap);
    long long cnt = std::min<long long>(avail, cap);
    for (long long i = 0; i < cnt; ++i) out[i] = h[(t - cnt + i) % kLossCap];
    *n = int(cnt);
    return CRV_OK;
  }

  crv_status gram_solve_host(const double* res, double* q) override {
    const size_t m = g.m, mp = g.mp, nk = g.dim == 3 ? m : 1;
    std::vector<double> pad(size_t(ipow(g.mp, g.dim)), 0.0);
    for (size_t k = 0; k < nk; ++k)
      for (size_t j = 0; j < m; ++j)
        for (size_t i = 0; i < m; ++i) pad[(k * mp + j) * mp + i] = res[(k * m + j) * m + i];
    crv_status s = upload(b.res, pad.data(), pad.size());
    if (s) return s;
    gram_solve();
    if ((s = check_launch())) return s;
    if ((s = download(pad.data(), b.q, pad.size()))) return s;
    for (size_t k = 0; k < nk; ++k)
      for (size_t j = 0; j < m; ++j)
        for (size_t i = 0; i < m; ++i) q[(k * m + j) * m + i] = pad[(k * mp + j) * mp + i];
    return CRV_OK;
  }

  crv_status mass_solve_host(const double* bin, double* x) override {
    crv_status s = upload(b.bvec, bin, nc);
    if (s) return s;
    mass_solve(b.bvec, b.bvec);
    if ((s = check_launch())) return s;
    return download(x, b.bvec, nc);
  }

  crv_status project_host(double* p) override {
    project_into_p();
    crv_status s = check_launch();
    if (s) return s;
    return download(p, b.p, nc);
  }
};

}  // namespace crv

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
struct crv_ctx {
  std::unique_ptr<crv::SolverBase> impl;
};

using namespace crv;

template <typename Real>
static crv_status make_solver(const crv_config* c, void* ws, std::unique_ptr<SolverBase>& out) {
  auto sv = std::make_unique<Solver<Real>>();
  Carve cv(ws);
  carve<Real>(cv, *c, sv->b);
  out = std::move(sv);
  return CRV_OK;
}


extern "C" {

const char* crv_last_error(void) { return g_err.c_str(); }

crv_status crv_config_default(crv_config* c) {
  if (!c) return fail(CRV_EINVAL, "config is NULL");
  std::memset(c, 0, sizeof(*c));
  c->dim = 2;
  c->n_elem = 32;
  c->degree = 2;
  c->width = 32;
  c->hidden = 3;
  c->precision = CRV_PREC_FP32;
  c->mu_w = 1.0;
  c->mu_g = 0.1;
  c->relperm_exp = 2.0;
  c->lr = 1e-4;
  c->beta1 = 0.9;
  c->beta2 = 0.999;
  c->eps = 1e-8;
  c->adam_iters = 100;
  c->substeps = 10;
  c->well_radius = 0.06;
  return CRV_OK;
}

crv_status crv_param_count(const crv_config* c, int64_t* n) {
  crv_status s = validate_config(c);
  if (s) return s;
  if (!n) return fail(CRV_EINVAL, "output is NULL");
  *n = mlp_param_count(c->dim, c->width, c->hidden);
  return CRV_OK;
}

crv_status crv_workspace_size(const crv_config* c, size_t* bytes) {
  crv_status s = validate_config(c);
  if (s) return s;
  if (!bytes) return fail(CRV_EINVAL, "output is NULL");
  Carve dry(nullptr);
  if (c->precision == CRV_PREC_FP64) {
    Buffers<double> b;
    *bytes = carve<double>(dry, *c, b);
  } else {
    Buffers<float> b;
    *bytes = carve<float>(dry, *c, b);
  }
  return CRV_OK;
}

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014), as a counter-based stream: output k of the
// generator started at state seed
static uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// seeded default parameters: Xavier-uniform weights a (2 u_k - 1),
// a = sqrt(6 / (fan_in + fan_out)), u_k = (output k >> 11) 2^-53 with k
// counting the weights in layout order; zero biases
static std::vector<double> default_theta(const crv_config& c, uint64_t seed) {
  std::vector<double> th;
  std::vector<int> d{c.dim};
  for (int l = 0; l < c.hidden; ++l) d.push_back(c.width);
  d.push_back(1);
  uint64_t k = 0;
  for (size_t l = 0; l + 1 < d.size(); ++l) {
    const double a = std::sqrt(6.0 / double(d[l] + d[l + 1]));
    for (int e = 0; e < d[l] * d[l + 1]; ++e) {
      const double u = double(splitmix64(seed, k++) >> 11) * 0x1.0p-53;
      th.push_back(a * (2.0 * u - 1.0));
    }
    th.insert(th.end(), size_t(d[l + 1]), 0.0);
  }
  return th;
}

crv_status crv_init(const crv_config* c, const double* log_perm, const double* porosity,
                    const crv_well* wells, int n_wells, const double* s0_coefs,
                    const double* theta0, uint64_t seed, void* d_workspace, size_t ws_bytes,
                    void* stream, crv_ctx** out) {
  static_assert(sizeof(crv_well) == 3 * sizeof(double), "crv_well is three doubles");
  crv_status s = validate_config(c);
  if (s) return s;
  if (!out || !log_perm || !porosity)
    return fail(CRV_EINVAL, "log_perm, porosity and out are required");
  std::vector<double> theta_default;
  if (!theta0) {
    theta_default = default_theta(*c, seed);
    theta0 = theta_default.data();
  }
  *out = nullptr;
  size_t need = 0;
  crv_workspace_size(c, &need);
  bool owns = false;
  if (d_workspace) {
    if (ws_bytes < need)
      return fail(CRV_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256)
      return fail(CRV_EINVAL, "workspace must be 256-byte aligned");
  } else {
    hipError_t e = hipMalloc(&d_workspace, need);
    if (e != hipSuccess) return fail(CRV_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    owns = true;
  }
  auto ctx = std::make_unique<crv_ctx>();
  if (c->precision == CRV_PREC_FP64)
    make_solver<double>(c, d_workspace, ctx->impl);
  else
    make_solver<float>(c, d_workspace, ctx->impl);
  SolverBase& sv = *ctx->impl;
  sv.cfg = *c;
  sv.g = make_geom(*c);
  sv.st = static_cast<hipStream_t>(stream);
  sv.P = mlp_param_count(c->dim, c->width, c->hidden);
  sv.ws = d_workspace;
  sv.owns_ws = owns;
  s = sv.init(log_perm, porosity, reinterpret_cast<const double*>(wells), n_wells, s0_coefs,
              theta0);
  if (s) return s;
  *out = ctx.release();
  return CRV_OK;
}

#define CRV_CTX(c)                                          \
  if (!(c) || !(c)->impl) return fail(CRV_EINVAL, "context is NULL"); \
  SolverBase& sv = *(c)->impl;

crv_status crv_pretrain_pressure(crv_ctx* c, int iters, double* final_loss) {
  CRV_CTX(c);
  if (iters < 0) return fail(CRV_EINVAL, "iters must be >= 0");
  crv_status s = sv.train(iters);
  if (s) return s;
  if (final_loss) {
    int n = 0;
    s = sv.loss_history(final_loss, 1, &n);
    if (s) return s;
    if (n == 0) *final_loss = NAN;
    if (n > 0 && !std::isfinite(*final_loss)) return fail(CRV_ENUMERIC, "non-finite loss");
  } else {
    hipError_t e = hipStreamSynchronize(sv.st);
    if (e != hipSuccess) return fail(CRV_EHIP, hipGetErrorString(e));
  }
  return CRV_OK;
}

crv_status crv_pressure_galerkin(crv_ctx* c, int max_iters, double rtol, int precond,
                                 double* p_coefs, int* iters, double* rel_residual) {
  CRV_CTX(c);
  return sv.pressure_galerkin(max_iters, rtol, precond, p_coefs, iters, rel_residual);
}

crv_status crv_step_galerkin(crv_ctx* c, double dt, int max_iters, double rtol, int precond,
                             int* iters, double* rel_residual) {
  CRV_CTX(c);
  return sv.step_galerkin(dt, max_iters, rtol, precond, iters, rel_residual);
}

crv_status crv_train_async(crv_ctx* c, int iters) {
  CRV_CTX(c);
  if (iters < 0) return fail(CRV_EINVAL, "iters must be >= 0");
  return sv.train(iters);
}

crv_status crv_sync(crv_ctx* c) {
  CRV_CTX(c);
  return sv.sync();
}

crv_status crv_step(crv_ctx* c, double dt) {
  CRV_CTX(c);
  if (!sv.pretrained) return fail(CRV_ESTATE, "crv_step before crv_pretrain_pressure");
  return sv.step(dt);
}

static crv_status step_batch(crv_ctx* const* ctxs, const double* dts, int n, int part) {
  if (n < 0 || (n > 0 && (!ctxs || !dts))) return fail(CRV_EINVAL, "bad batch arrays");
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !ctxs[i]->impl) return fail(CRV_EINVAL, "context is NULL");
    if (!(dts[i] > 0) || !std::isfinite(dts[i])) return fail(CRV_EINVAL, "dt must be > 0");
    if (!ctxs[i]->impl->pretrained) return fail(CRV_ESTATE, "crv_step_batch before crv_pretrain_pressure");
  }
  // one batched launch per kernel when every context has the first one's
  // configuration and the workspaces lie at one stride, in order, without
  // overlap; otherwise each context steps on its own stream
  if (n >= 2) {
    SolverBase& s0 = *ctxs[0]->impl;
    const char* base = static_cast<const char*>(s0.ws);
    const int64_t zb = static_cast<const char*>(ctxs[1]->impl->ws) - base;
    size_t need = 0;
    crv_workspace_size(&s0.cfg, &need);
    bool ok = s0.batchable() && zb > 0 && uint64_t(zb) >= need;
    for (int i = 1; ok && i < n; ++i) {
      SolverBase& si = *ctxs[i]->impl;
      ok = si.batchable() && same_config(si.cfg, s0.cfg) && si.batch_tag() == s0.batch_tag() &&
           static_cast<const char*>(si.ws) == base + int64_t(i) * zb;
    }
    if (ok) {
      std::vector<SolverBase*> all(static_cast<size_t>(n));
      for (int i = 0; i < n; ++i) all[size_t(i)] = ctxs[i]->impl.get();
      return s0.step_batched(all.data(), dts, n, zb, part);
    }
  }
  for (int i = 0; i < n; ++i) {
    const crv_status s = ctxs[i]->impl->step(dts[i]);
    if (s) return s;
  }
  return CRV_OK;
}

crv_status crv_step_batch(crv_ctx* const* ctxs, const double* dts, int n) {
  return step_batch(ctxs, dts, n, 0);
}

crv_status crv_step_batch_shared(crv_ctx* const* ctxs, const double* dts, int n) {
  return step_batch(ctxs, dts, n, 1);
}

crv_status crv_step_batch_shared_part(crv_ctx* const* ctxs, const double* dts, int n, int part) {
  if (part < 1 || part > 16) return fail(CRV_EINVAL, "part must be in [1, 16]");
  return step_batch(ctxs, dts, n, part);
}

crv_status crv_get_fields(crv_ctx* c, double* p_nodal, double* s_coefs, double* s_nodal) {
  CRV_CTX(c);
  return sv.fields(p_nodal, s_coefs, s_nodal);
}

crv_status crv_loss_grad(crv_ctx* c, double* loss, double* dtheta, double* dlogperm) {
  CRV_CTX(c);
  return sv.loss_grad(loss, dtheta, dlogperm);
}

crv_status crv_loss_grad_device(crv_ctx* c, double* d_loss, float* d_dtheta, float* d_dlogperm) {
  CRV_CTX(c);
  return sv.loss_grad_device(d_loss, d_dtheta, d_dlogperm);
}

crv_status crv_set_params_device(crv_ctx* c, const float* d_theta, const float* d_log_perm) {
  CRV_CTX(c);
  return sv.set_params_device(d_theta, d_log_perm);
}

crv_status crv_get_state(crv_ctx* c, double* theta, double* m, double* v, int64_t* t) {
  CRV_CTX(c);
  return sv.get_state(theta, m, v, t);
}

crv_status crv_set_state(crv_ctx* c, const double* theta, const double* m, const double* v,
                         int64_t t) {
  CRV_CTX(c);
  return sv.set_state(theta, m, v, t);
}

crv_status crv_set_saturation(crv_ctx* c, const double* s_coefs) {
  CRV_CTX(c);
  if (!s_coefs) return fail(CRV_EINVAL, "s_coefs is NULL");
  return sv.set_saturation(s_coefs);
}

crv_status crv_set_log_perm(crv_ctx* c, const double* log_perm) {
  CRV_CTX(c);
  if (!log_perm) return fail(CRV_EINVAL, "log_perm is NULL");
  return sv.set_log_perm(log_perm);
}

crv_status crv_set_observations(crv_ctx* c, const double* data, const double* weights) {
  CRV_CTX(c);
  if (data && !weights) return fail(CRV_EINVAL, "weights are required with data");
  return sv.set_observations(data, weights);
}

crv_status crv_invert(crv_ctx* c, int iters, double lr_logk) {
  CRV_CTX(c);
  return sv.invert(iters, lr_logk);
}

crv_status crv_get_log_perm(crv_ctx* c, double* log_perm) {
  CRV_CTX(c);
  if (!log_perm) return fail(CRV_EINVAL, "log_perm is NULL");
  return sv.get_log_perm(log_perm);
}

crv_status crv_loss_history(crv_ctx* c, double* out, int cap, int* n) {
  CRV_CTX(c);
  if (!out || !n || cap < 0) return fail(CRV_EINVAL, "bad output buffer");
  return sv.loss_history(out, cap, n);
}

crv_status crv_gram_solve(crv_ctx* c, const double* res, double* q) {
  CRV_CTX(c);
  if (!res || !q) return fail(CRV_EINVAL, "NULL array");
  return sv.gram_solve_host(res, q);
}

crv_status crv_mass_solve(crv_ctx* c, const double* b, double* x) {
  CRV_CTX(c);
  if (!b || !x) return fail(CRV_EINVAL, "NULL array");
  return sv.mass_solve_host(b, x);
}

crv_status crv_project_pressure(crv_ctx* c, double* p) {
  CRV_CTX(c);
  if (!p) return fail(CRV_EINVAL, "NULL array");
  return sv.project_host(p);
}

crv_status crv_saturation_substeps(crv_ctx* c, double tau, int n) {
  CRV_CTX(c);
  return sv.substeps(tau, n);
}

crv_status crv_profile_enable(crv_ctx* c, int enable) {
  CRV_CTX(c);
  hipError_t e = hipStreamSynchronize(sv.st);
  if (e != hipSuccess) return fail(CRV_EHIP, hipGetErrorString(e));
  sv.profile_reset();
  sv.prof = enable != 0;
  return CRV_OK;
}

crv_status crv_profile_read(crv_ctx* c, int kernel, double* total_ms, int64_t* count) {
  CRV_CTX(c);
  if (kernel < 0 || kernel >= CRV_K_COUNT || !total_ms || !count)
    return fail(CRV_EINVAL, "bad kernel id or output");
  hipError_t e = hipStreamSynchronize(sv.st);
  if (e != hipSuccess) return fail(CRV_EHIP, hipGetErrorString(e));
  double tot = 0;
  int64_t n = 0;
  for (auto& m : sv.marks) {
    if (m.first != kernel) continue;
    float ms = 0;
    e = hipEventElapsedTime(&ms, m.second.first, m.second.second);
    if (e != hipSuccess) return fail(CRV_EHIP, hipGetErrorString(e));
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *count = n;
  return CRV_OK;
}

crv_status crv_destroy(crv_ctx* c) {
  if (!c) return CRV_OK;
  if (c->impl) (void)hipStreamSynchronize(c->impl->st);
  delete c;
  return CRV_OK;
}

}  // extern "C"
