// Host-only driver of the C ABI's argument and configuration checks, built
// with AddressSanitizer and UndefinedBehaviorSanitizer on the host code of
// the library (python -m paper_2604_20731_amd.build --sanitize).  It runs
// without a GPU: every call below must return its documented status before
// (or instead of) any device work, and the sanitizers must stay silent.
// Prints one line per check and exits non-zero on the first wrong status.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/crv.h"

static int g_fail = 0;

static void expect(const char* what, crv_status got, crv_status want) {
  const bool ok = got == want;
  std::printf("%s %-58s status %d (want %d)%s%s\n", ok ? "ok  " : "FAIL", what, int(got), int(want),
              ok ? "" : " : ", ok ? "" : crv_last_error());
  if (!ok) g_fail = 1;
}

int main() {
  crv_config c;
  expect("config_default", crv_config_default(&c), CRV_OK);
  expect("config_default(NULL)", crv_config_default(nullptr), CRV_EINVAL);

  size_t bytes = 0;
  expect("workspace_size default", crv_workspace_size(&c, &bytes), CRV_OK);
  expect("workspace_size NULL out", crv_workspace_size(&c, nullptr), CRV_EINVAL);
  expect("workspace_size NULL config", crv_workspace_size(nullptr, &bytes), CRV_EINVAL);
  int64_t np = 0;
  expect("param_count", crv_param_count(&c, &np), CRV_OK);

  // every field out of range, one at a time
  struct Bad {
    const char* name;
    void (*set)(crv_config*);
  };
  const Bad bad[] = {
      {"dim 4", [](crv_config* x) { x->dim = 4; }},
      {"n_elem 2", [](crv_config* x) { x->n_elem = 2; }},
      {"n_elem 2000", [](crv_config* x) { x->n_elem = 2000; }},
      {"3D n_elem 300", [](crv_config* x) { x->dim = 3; x->n_elem = 300; x->hidden = 4; }},
      {"degree 0", [](crv_config* x) { x->degree = 0; }},
      {"width 48", [](crv_config* x) { x->width = 48; }},
      {"hidden 9", [](crv_config* x) { x->hidden = 9; }},
      {"precision 9", [](crv_config* x) { x->precision = 9; }},
      {"precision -1", [](crv_config* x) { x->precision = -1; }},
      {"bf16 width 16", [](crv_config* x) { x->precision = CRV_PREC_BF16; x->width = 16; }},
      {"mu_g 0", [](crv_config* x) { x->mu_g = 0.0; }},
      {"mu_w NaN", [](crv_config* x) { x->mu_w = NAN; }},
      {"relperm_exp 0.5", [](crv_config* x) { x->relperm_exp = 0.5; }},
      {"lr -1", [](crv_config* x) { x->lr = -1.0; }},
      {"beta1 1", [](crv_config* x) { x->beta1 = 1.0; }},
      {"eps -1", [](crv_config* x) { x->eps = -1.0; }},
      {"adam_iters -1", [](crv_config* x) { x->adam_iters = -1; }},
      {"substeps 0", [](crv_config* x) { x->substeps = 0; }},
      {"well_radius 0", [](crv_config* x) { x->well_radius = 0.0; }},
      {"gravity -1", [](crv_config* x) { x->gravity = -1.0; }},
      {"rho_g inf", [](crv_config* x) { x->rho_g = INFINITY; }},
      {"boundary_factor 2", [](crv_config* x) { x->boundary_factor = 2; }},
  };
  for (const Bad& b : bad) {
    crv_config x;
    crv_config_default(&x);
    b.set(&x);
    char what[96];
    std::snprintf(what, sizeof what, "workspace_size %s", b.name);
    expect(what, crv_workspace_size(&x, &bytes), CRV_EINVAL);
    std::snprintf(what, sizeof what, "init %s", b.name);
    crv_ctx* ctx = nullptr;
    std::vector<double> one(64, 0.0);
    expect(what, crv_init(&x, one.data(), one.data(), nullptr, 0, nullptr, one.data(), 0, nullptr, 0,
                          nullptr, &ctx),
           CRV_EINVAL);
  }

  // missing arrays, and a workspace that is too small or misaligned
  crv_ctx* ctx = nullptr;
  const size_t nn = size_t(c.n_elem + 1) * (c.n_elem + 1);
  std::vector<double> lp(nn, 0.0), po(nn, 0.2), th(size_t(np), 0.0);
  expect("init NULL log_perm", crv_init(&c, nullptr, po.data(), nullptr, 0, nullptr, th.data(),
                                        0, nullptr, 0, nullptr, &ctx), CRV_EINVAL);
  expect("init NULL out", crv_init(&c, lp.data(), po.data(), nullptr, 0, nullptr, th.data(),
                                   0, nullptr, 0, nullptr, nullptr), CRV_EINVAL);
  alignas(256) static char small[512];
  expect("init workspace too small", crv_init(&c, lp.data(), po.data(), nullptr, 0, nullptr,
                                              th.data(), 0, small, sizeof small, nullptr, &ctx),
         CRV_ENOMEM);
  expect("init workspace misaligned", crv_init(&c, lp.data(), po.data(), nullptr, 0, nullptr,
                                               th.data(), 0, small + 8, size_t(1) << 40, nullptr,
                                               &ctx),
         CRV_EINVAL);

  // calls on a missing context
  double d = 0.0;
  int it = 0;
  int64_t cnt = 0;
  expect("pretrain NULL", crv_pretrain_pressure(nullptr, 1, &d), CRV_EINVAL);
  expect("train_async NULL", crv_train_async(nullptr, 1), CRV_EINVAL);
  expect("sync NULL", crv_sync(nullptr), CRV_EINVAL);
  expect("step NULL", crv_step(nullptr, 1e-3), CRV_EINVAL);
  expect("get_fields NULL", crv_get_fields(nullptr, &d, &d, &d), CRV_EINVAL);
  expect("loss_grad NULL", crv_loss_grad(nullptr, &d, &d, &d), CRV_EINVAL);
  expect("get_state NULL", crv_get_state(nullptr, &d, &d, &d, &cnt), CRV_EINVAL);
  expect("set_state NULL", crv_set_state(nullptr, &d, &d, &d, 0), CRV_EINVAL);
  expect("set_saturation NULL", crv_set_saturation(nullptr, &d), CRV_EINVAL);
  expect("set_log_perm NULL", crv_set_log_perm(nullptr, &d), CRV_EINVAL);
  float fd = 0;
  expect("loss_grad_device NULL", crv_loss_grad_device(nullptr, &d, &fd, &fd), CRV_EINVAL);
  expect("set_params_device NULL", crv_set_params_device(nullptr, &fd, &fd), CRV_EINVAL);
  expect("loss_history NULL", crv_loss_history(nullptr, &d, 1, &it), CRV_EINVAL);
  expect("gram_solve NULL", crv_gram_solve(nullptr, &d, &d), CRV_EINVAL);
  expect("mass_solve NULL", crv_mass_solve(nullptr, &d, &d), CRV_EINVAL);
  expect("project_pressure NULL", crv_project_pressure(nullptr, &d), CRV_EINVAL);
  expect("saturation_substeps NULL", crv_saturation_substeps(nullptr, 1e-3, 1), CRV_EINVAL);
  expect("pressure_galerkin NULL", crv_pressure_galerkin(nullptr, 10, 1e-6, 1, &d, &it, &d),
         CRV_EINVAL);
  expect("step_galerkin NULL", crv_step_galerkin(nullptr, 1e-3, 10, 1e-6, 1, &it, &d), CRV_EINVAL);
  expect("set_observations NULL", crv_set_observations(nullptr, &d, &d), CRV_EINVAL);
  expect("invert NULL", crv_invert(nullptr, 1, 1e-3), CRV_EINVAL);
  expect("get_log_perm NULL", crv_get_log_perm(nullptr, &d), CRV_EINVAL);
  expect("profile_enable NULL", crv_profile_enable(nullptr, 1), CRV_EINVAL);
  expect("profile_read NULL", crv_profile_read(nullptr, 0, &d, &cnt), CRV_EINVAL);
  expect("destroy NULL", crv_destroy(nullptr), CRV_OK);

  // batches
  expect("step_batch n < 0", crv_step_batch(nullptr, nullptr, -1), CRV_EINVAL);
  expect("step_batch NULL arrays", crv_step_batch(nullptr, nullptr, 2), CRV_EINVAL);
  crv_ctx* none[2] = {nullptr, nullptr};
  const double dts[2] = {1e-3, 1e-3};
  expect("step_batch NULL context", crv_step_batch(none, dts, 2), CRV_EINVAL);
  expect("step_batch empty", crv_step_batch(nullptr, nullptr, 0), CRV_OK);
  expect("step_batch_shared NULL context", crv_step_batch_shared(none, dts, 2), CRV_EINVAL);
  expect("step_batch_shared_part NULL context", crv_step_batch_shared_part(none, dts, 2, 2), CRV_EINVAL);
  expect("step_batch_shared_part part 0", crv_step_batch_shared_part(none, dts, 2, 0), CRV_EINVAL);
  expect("step_batch_shared_part part 17", crv_step_batch_shared_part(none, dts, 2, 17), CRV_EINVAL);

  // the allocation-free Gram solve: sizes beyond its array, missing arrays
  float f = 0.f;
  expect("gram_solve_noalloc n_elem 513", crv_gram_solve_noalloc(513, &f, &f, nullptr, nullptr),
         CRV_EINVAL);
  expect("gram_solve_noalloc n_elem 3", crv_gram_solve_noalloc(3, &f, &f, nullptr, nullptr),
         CRV_EINVAL);
  expect("gram_solve_noalloc NULL res", crv_gram_solve_noalloc(64, nullptr, &f, nullptr, nullptr),
         CRV_EINVAL);

  if (std::strlen(crv_last_error()) == 0) {
    std::printf("FAIL crv_last_error is empty after an error\n");
    g_fail = 1;
  }
  std::printf(g_fail ? "abi_check: FAILED\n" : "abi_check: all checks passed\n");
  return g_fail;
}
