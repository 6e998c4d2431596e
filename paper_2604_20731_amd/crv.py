"""ctypes binding of libcrv (include/crv.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
to float64 host buffers, allocates the device workspace with torch (device
memory and the stream are the only things torch provides) and checks status
codes.  Importing it fails loudly when libcrv.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrv.so")

CRV_OK, CRV_EINVAL, CRV_ENOMEM, CRV_EHIP, CRV_ENUMERIC, CRV_ESTATE = 0, -1, -2, -3, -4, -5
PREC = {"fp32": 0, "bf16": 1, "fp64": 2, "bf16x3": 3, "bf16x3f": 4}
PRECOND = {"jacobi": 0, "kron": 1}  # CRV_PRECOND_* of the Galerkin CG
STATUS_NAMES = {0: "CRV_OK", -1: "CRV_EINVAL", -2: "CRV_ENOMEM", -3: "CRV_EHIP",
                -4: "CRV_ENUMERIC", -5: "CRV_ESTATE"}

EXPORTED = [
    "crv_config_default", "crv_param_count", "crv_workspace_size", "crv_init",
    "crv_pretrain_pressure", "crv_train_async", "crv_sync", "crv_step", "crv_step_batch",
    "crv_step_batch_shared", "crv_step_batch_shared_part",
    "crv_get_fields", "crv_loss_grad", "crv_loss_grad_device", "crv_set_params_device",
    "crv_get_state", "crv_set_state", "crv_set_saturation", "crv_set_log_perm", "crv_loss_history",
    "crv_set_observations", "crv_invert", "crv_get_log_perm",
    "crv_gram_solve", "crv_gram_solve_noalloc", "crv_mass_solve", "crv_project_pressure",
    "crv_saturation_substeps", "crv_pressure_galerkin", "crv_step_galerkin",
    "crv_profile_enable", "crv_profile_read", "crv_destroy", "crv_last_error",
]

KERNELS = ["mlp_fwd", "mlp_bwd", "residual", "gram_dst", "gram_lines", "adjoint", "loss",
           "grad_reduce", "adam", "refresh", "project", "ads_assemble", "mass_rows", "mass_cols"]


class CrvConfig(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n_elem", C.c_int), ("degree", C.c_int), ("width", C.c_int),
        ("hidden", C.c_int), ("precision", C.c_int),
        ("mu_w", C.c_double), ("mu_g", C.c_double), ("relperm_exp", C.c_double),
        ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
        ("adam_iters", C.c_int), ("substeps", C.c_int), ("well_radius", C.c_double),
        ("gravity", C.c_double), ("rho_w", C.c_double), ("rho_g", C.c_double),
        ("boundary_factor", C.c_int),
    ]


class CrvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load() -> C.CDLL:
    # torch carries its own copy of the HIP runtime; loading it first makes
    # libcrv bind to that same copy (one runtime per process), which the
    # torch-allocated workspace and streams require.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libcrv.so is not built ({LIB_PATH}); run "
                          "python -m paper_2604_20731_amd.build")
    lib = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    cfgp = C.POINTER(CrvConfig)
    vp = C.c_void_p
    sig = {
        "crv_config_default": [cfgp],
        "crv_param_count": [cfgp, C.POINTER(C.c_int64)],
        "crv_workspace_size": [cfgp, C.POINTER(C.c_size_t)],
        "crv_init": [cfgp, dp, dp, dp, C.c_int, dp, dp, C.c_uint64, vp, C.c_size_t, vp,
                     C.POINTER(vp)],
        "crv_pretrain_pressure": [vp, C.c_int, dp],
        "crv_step": [vp, C.c_double],
        "crv_step_batch": [C.POINTER(vp), dp, C.c_int],
        "crv_step_batch_shared": [C.POINTER(vp), dp, C.c_int],
        "crv_step_batch_shared_part": [C.POINTER(vp), dp, C.c_int, C.c_int],
        "crv_train_async": [vp, C.c_int],
        "crv_sync": [vp],
        "crv_get_fields": [vp, dp, dp, dp],
        "crv_loss_grad": [vp, dp, dp, dp],
        "crv_loss_grad_device": [vp, vp, vp, vp],
        "crv_set_params_device": [vp, vp, vp],
        "crv_get_state": [vp, dp, dp, dp, C.POINTER(C.c_int64)],
        "crv_set_state": [vp, dp, dp, dp, C.c_int64],
        "crv_set_saturation": [vp, dp],
        "crv_set_log_perm": [vp, dp],
        "crv_loss_history": [vp, dp, C.c_int, C.POINTER(C.c_int)],
        "crv_set_observations": [vp, dp, dp],
        "crv_invert": [vp, C.c_int, C.c_double],
        "crv_get_log_perm": [vp, dp],
        "crv_gram_solve": [vp, dp, dp],
        "crv_gram_solve_noalloc": [C.c_int, vp, vp, vp, vp],
        "crv_mass_solve": [vp, dp, dp],
        "crv_project_pressure": [vp, dp],
        "crv_saturation_substeps": [vp, C.c_double, C.c_int],
        "crv_pressure_galerkin": [vp, C.c_int, C.c_double, C.c_int, dp, C.POINTER(C.c_int), dp],
        "crv_step_galerkin": [vp, C.c_double, C.c_int, C.c_double, C.c_int, C.POINTER(C.c_int),
                              dp],
        "crv_profile_enable": [vp, C.c_int],
        "crv_profile_read": [vp, C.c_int, dp, C.POINTER(C.c_int64)],
        "crv_destroy": [vp],
        "crv_last_error": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_char_p if name == "crv_last_error" else C.c_int
    return lib


LIB = _load()


def _check(status: int):
    if status != CRV_OK:
        raise CrvError(status, LIB.crv_last_error().decode())


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def config(dim=2, n_elem=32, degree=2, width=32, hidden=3, precision="fp32", **kw) -> CrvConfig:
    c = CrvConfig()
    _check(LIB.crv_config_default(C.byref(c)))
    c.dim, c.n_elem, c.degree, c.width, c.hidden = dim, n_elem, degree, width, hidden
    c.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


def param_count(cfg: CrvConfig) -> int:
    n = C.c_int64()
    _check(LIB.crv_param_count(C.byref(cfg), C.byref(n)))
    return n.value


def workspace_size(cfg: CrvConfig) -> int:
    n = C.c_size_t()
    _check(LIB.crv_workspace_size(C.byref(cfg), C.byref(n)))
    return n.value


class Scenario:
    """One reservoir scenario: a libcrv context on the current torch stream
    with a torch-allocated device workspace (or the given uint8 device tensor
    of at least workspace_size(cfg) bytes, 256-byte aligned).  theta0 None
    takes the library's seeded default parameters (seed)."""

    def __init__(self, cfg: CrvConfig, log_perm, porosity, wells, theta0, s0_coefs=None,
                 device: str = "cuda:0", stream=None, workspace=None, seed: int = 0):
        import torch  # device memory and streams only
        self.cfg = cfg
        self.dim, self.ne, self.r = cfg.dim, cfg.n_elem, cfg.degree
        self.nn = (self.ne + 1) ** self.dim
        self.nb = self.ne + self.r
        self.nc = self.nb ** self.dim
        self.m = self.ne - 1
        self.P = param_count(cfg)
        self.ws_bytes = workspace_size(cfg)
        if workspace is None:
            self._ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        else:
            if workspace.dtype != torch.uint8 or workspace.numel() < self.ws_bytes:
                raise ValueError(f"workspace must be a uint8 tensor of >= {self.ws_bytes} bytes")
            self._ws = workspace
        st = stream if stream is not None else torch.cuda.current_stream(self._ws.device)
        self._stream = st
        lp, po = _f64(log_perm).ravel(), _f64(porosity).ravel()
        w = _f64(wells).reshape(-1, 3)
        th = None if theta0 is None else _f64(theta0).ravel()
        s0 = None if s0_coefs is None else _f64(s0_coefs).ravel()
        if lp.size != self.nn or po.size != self.nn:
            raise ValueError("nodal arrays must have (N+1)^d entries")
        if th is not None and th.size != self.P:
            raise ValueError(f"theta0 must have {self.P} entries")
        if s0 is not None and s0.size != self.nc:
            raise ValueError("s0_coefs must have nb^d entries")
        ctx = C.c_void_p()
        _check(LIB.crv_init(C.byref(cfg), _dp(lp), _dp(po), _dp(w), int(w.shape[0]), _dp(s0),
                            _dp(th), int(seed), C.c_void_p(self._ws.data_ptr()), self.ws_bytes,
                            C.c_void_p(st.cuda_stream), C.byref(ctx)))
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            LIB.crv_destroy(self.ctx)
            self.ctx = None
        self._ws = None  # the workspace may be reused once the context is gone

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- algorithm calls ------------------------------------------------------
    def pretrain_pressure(self, iters: int) -> float:
        out = C.c_double()
        _check(LIB.crv_pretrain_pressure(self.ctx, int(iters), C.byref(out)))
        return out.value

    def step(self, dt: float):
        _check(LIB.crv_step(self.ctx, float(dt)))

    def train_async(self, iters: int):
        _check(LIB.crv_train_async(self.ctx, int(iters)))

    def sync(self):
        _check(LIB.crv_sync(self.ctx))

    @property
    def stream(self):
        return self._stream

    def fields(self):
        shp_n = (self.ne + 1,) * self.dim
        shp_c = (self.nb,) * self.dim
        p = np.empty(shp_n)
        sc = np.empty(shp_c)
        sn = np.empty(shp_n)
        _check(LIB.crv_get_fields(self.ctx, _dp(p), _dp(sc), _dp(sn)))
        return p, sc, sn

    def loss_grad(self, with_logperm: bool = False):
        loss = C.c_double()
        g = np.empty(self.P)
        gl = np.empty((self.ne + 1,) * self.dim) if with_logperm else None
        _check(LIB.crv_loss_grad(self.ctx, C.byref(loss), _dp(g), _dp(gl)))
        return (loss.value, g, gl) if with_logperm else (loss.value, g)

    @staticmethod
    def _device_f32(t, n: int, name: str):
        import torch
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
        return C.c_void_p(t.data_ptr())

    def set_params_device(self, theta=None, log_perm=None):
        """crv_set_params_device: theta and/or the nodal log K from float32
        CUDA tensors, read in order on this scenario's stream after the
        work already queued on the current stream."""
        import torch
        cur = torch.cuda.current_stream(self._ws.device)
        self._stream.wait_stream(cur)
        th = None if theta is None else self._device_f32(theta, self.P, "theta")
        lk = None if log_perm is None else self._device_f32(log_perm, self.nn, "log_perm")
        for t in (theta, log_perm):
            if t is not None and self._stream != cur:
                t.record_stream(self._stream)
        _check(LIB.crv_set_params_device(self.ctx, th, lk))

    def loss_grad_device(self, with_logperm: bool = False):
        """crv_loss_grad_device: the loss (float64) and gradients (float32)
        as CUDA tensors, ready for work on the current stream; no host
        transfer and no wait."""
        import torch
        dev = self._ws.device
        cur = torch.cuda.current_stream(dev)
        loss = torch.empty((), dtype=torch.float64, device=dev)
        g = torch.empty(self.P, dtype=torch.float32, device=dev)
        gl = (torch.empty((self.ne + 1,) * self.dim, dtype=torch.float32, device=dev)
              if with_logperm else None)
        self._stream.wait_stream(cur)
        _check(LIB.crv_loss_grad_device(self.ctx, C.c_void_p(loss.data_ptr()),
                                        C.c_void_p(g.data_ptr()),
                                        None if gl is None else C.c_void_p(gl.data_ptr())))
        if self._stream != cur:
            for t in (loss, g, gl):
                if t is not None:
                    t.record_stream(self._stream)
            cur.wait_stream(self._stream)
        return (loss, g, gl) if with_logperm else (loss, g)

    def get_state(self):
        th, m, v = np.empty(self.P), np.empty(self.P), np.empty(self.P)
        t = C.c_int64()
        _check(LIB.crv_get_state(self.ctx, _dp(th), _dp(m), _dp(v), C.byref(t)))
        return th, m, v, t.value

    def set_state(self, theta, m=None, v=None, t=0):
        _check(LIB.crv_set_state(self.ctx, _dp(_f64(theta)), _dp(None if m is None else _f64(m)),
                                 _dp(None if v is None else _f64(v)), int(t)))

    def set_saturation(self, s_coefs):
        a = _f64(s_coefs).ravel()
        if a.size != self.nc:
            raise ValueError(f"s_coefs has {a.size} entries, expected {self.nc}")
        _check(LIB.crv_set_saturation(self.ctx, _dp(a)))

    def set_log_perm(self, log_perm):
        """Replace the nodal log-permeability; alpha follows."""
        a = _f64(log_perm).ravel()
        if a.size != self.nn:
            raise ValueError(f"log_perm has {a.size} entries, expected {self.nn}")
        _check(LIB.crv_set_log_perm(self.ctx, _dp(a)))

    def set_observations(self, data, weights):
        """Nodal pressure data and weights (>= 0) of the inverse problem;
        data None clears them."""
        if data is None:
            _check(LIB.crv_set_observations(self.ctx, None, None))
            return
        d, w = _f64(data).ravel(), _f64(weights).ravel()
        if d.size != self.nn or w.size != self.nn:
            raise ValueError(f"observations need {self.nn} nodal entries")
        _check(LIB.crv_set_observations(self.ctx, _dp(d), _dp(w)))

    def invert(self, iters: int, lr_logk: float):
        """crv_invert: joint Adam iterations on the network and log K."""
        _check(LIB.crv_invert(self.ctx, int(iters), float(lr_logk)))

    def log_perm(self) -> np.ndarray:
        out = np.empty((self.ne + 1,) * self.dim)
        _check(LIB.crv_get_log_perm(self.ctx, _dp(out)))
        return out

    def set_theta(self, theta):
        """Replace the network parameters, keeping the Adam moments and step count."""
        a = _f64(theta).ravel()
        if a.size != self.P:
            raise ValueError(f"theta has {a.size} entries, expected {self.P}")
        _check(LIB.crv_set_state(self.ctx, _dp(a), None, None, -1))

    def loss_history(self, cap: int = 1 << 16) -> np.ndarray:
        out = np.empty(cap)
        n = C.c_int()
        _check(LIB.crv_loss_history(self.ctx, _dp(out), cap, C.byref(n)))
        return out[: n.value].copy()

    def gram_solve(self, res):
        r = _f64(res)
        q = np.empty_like(r)
        _check(LIB.crv_gram_solve(self.ctx, _dp(r), _dp(q)))
        return q

    def mass_solve(self, b):
        bb = _f64(b)
        x = np.empty_like(bb)
        _check(LIB.crv_mass_solve(self.ctx, _dp(bb), _dp(x)))
        return x

    def project_pressure(self):
        p = np.empty((self.nb,) * self.dim)
        _check(LIB.crv_project_pressure(self.ctx, _dp(p)))
        return p

    def saturation_substeps(self, tau: float, n: int):
        _check(LIB.crv_saturation_substeps(self.ctx, float(tau), int(n)))

    def pressure_galerkin(self, max_iters: int = 20000, rtol: float = 1e-6,
                          precond: str = "kron"):
        """Galerkin pressure of the current saturation (2D) by CG with the
        preconditioner "kron" (scaled Kronecker inverse) or "jacobi":
        (coefficients nb^2, CG iterations, |r|/|F|)."""
        nb = self.cfg.n_elem + self.cfg.degree
        out = np.zeros(nb ** self.cfg.dim)
        it, rr = C.c_int(), C.c_double()
        _check(LIB.crv_pressure_galerkin(self.ctx, int(max_iters), float(rtol),
                                         PRECOND[precond], _dp(out), C.byref(it), C.byref(rr)))
        return out, it.value, rr.value

    def step_galerkin(self, dt: float, max_iters: int = 20000, rtol: float = 1e-6,
                      precond: str = "kron"):
        """Substeps with the current pressure coefficients, then the Galerkin
        pressure of the new saturation: (CG iterations, |r|/|F|)."""
        it, rr = C.c_int(), C.c_double()
        _check(LIB.crv_step_galerkin(self.ctx, float(dt), int(max_iters), float(rtol),
                                     PRECOND[precond], C.byref(it), C.byref(rr)))
        return it.value, rr.value

    def profile_enable(self, on: bool = True):
        _check(LIB.crv_profile_enable(self.ctx, 1 if on else 0))

    def profile_read(self):
        """{kernel name: (total ms, launches)} since the last profile_enable."""
        out = {}
        for k, name in enumerate(KERNELS):
            ms, n = C.c_double(), C.c_int64()
            _check(LIB.crv_profile_read(self.ctx, k, C.byref(ms), C.byref(n)))
            out[name] = (ms.value, n.value)
        return out


def gram_solve_noalloc(n_elem: int, res, q, loss=None, stream=None):
    """crv_gram_solve_noalloc: q = G^-1 res (2D) on device tensors with no
    allocation.  res, q: contiguous float32 CUDA tensors of (n_elem-1)^2
    entries; loss (optional): a float64 CUDA tensor of one entry that
    receives res . q.  Enqueued on stream (default: the current torch
    stream); returns without waiting."""
    import torch
    m2 = (int(n_elem) - 1) ** 2
    for name, t, dt in (("res", res, torch.float32), ("q", q, torch.float32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() != m2:
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of {m2} entries")
    if loss is not None and (loss.dtype != torch.float64 or not loss.is_cuda or loss.numel() != 1):
        raise ValueError("loss must be a float64 CUDA tensor of one entry")
    st = stream if stream is not None else torch.cuda.current_stream(res.device)
    _check(LIB.crv_gram_solve_noalloc(int(n_elem), C.c_void_p(res.data_ptr()),
                                      C.c_void_p(q.data_ptr()),
                                      None if loss is None else C.c_void_p(loss.data_ptr()),
                                      C.c_void_p(st.cuda_stream)))


def step_batch(scenarios, dts, shared: bool = False, part: int = 1):
    """crv_step_batch: one coupled step for each scenario, bitwise the results
    of one crv_step each.  Scenarios of one configuration whose workspaces lie
    at one stride (a Bucket, or a run of consecutive scenarios of one) step
    with one launch per kernel; others each on their own stream, with no
    host wait between them.  shared: crv_step_batch_shared (the batched
    backward shares the device's blocks among the scenarios: faster, equal to
    rounding); part > 1: crv_step_batch_shared_part (the batch's backward
    takes 1/part of the device's blocks, for batches stepped on several
    streams at once)."""
    n = len(scenarios)
    if len(dts) != n:
        raise ValueError("one dt per scenario")
    ctxs = (C.c_void_p * n)(*[sc.ctx for sc in scenarios])
    d = _f64(dts)
    if shared and part != 1:
        _check(LIB.crv_step_batch_shared_part(ctxs, _dp(d), n, int(part)))
        return
    fn = LIB.crv_step_batch_shared if shared else LIB.crv_step_batch
    _check(fn(ctxs, _dp(d), n))


class Bucket:
    """Scenarios of one configuration whose workspaces lie at a fixed stride
    in one device allocation, so that crv_step_batch advances them with one
    launch per kernel of the coupled step (the scenario index selects the
    workspace).  All of them run on one stream."""

    def __init__(self, cfg: CrvConfig, problems, device: str = "cuda:0", stream=None):
        import torch  # device memory and streams only
        self.cfg = cfg
        self.stride = (workspace_size(cfg) + 255) // 256 * 256
        n = len(problems)
        self._mem = torch.empty(self.stride * n + 256, dtype=torch.uint8, device=device)
        lead = (-self._mem.data_ptr()) % 256
        st = stream if stream is not None else torch.cuda.current_stream(self._mem.device)
        self.scenarios = [
            Scenario(cfg, p.log_perm, p.porosity, p.wells, p.theta0, p.s0_coefs, device=device,
                     stream=st, workspace=self._mem[lead + k * self.stride:
                                                    lead + (k + 1) * self.stride])
            for k, p in enumerate(problems)]

    def step(self, dts, shared: bool = False, part: int = 1):
        step_batch(self.scenarios, dts, shared, part)

    def close(self):
        for sc in self.scenarios:
            sc.close()
        self.scenarios = []
        self._mem = None


class BucketGroup:
    """Scenarios of one configuration split into `groups` Buckets, each on its
    own stream, stepped together: every bucket's batched step is enqueued on
    its stream with no host wait, so one bucket's forward and small kernels
    run beside another's backward.  With shared=True each bucket's backward
    takes 1/part of the device's blocks (crv_step_batch_shared_part), leaving
    room for the others; part = 1 gives each the whole device."""

    def __init__(self, cfg: CrvConfig, problems, groups: int = 4, device: str = "cuda:0"):
        import torch  # device memory and streams only
        problems = list(problems)
        if groups < 1:
            raise ValueError("groups must be >= 1")
        per = (len(problems) + groups - 1) // groups
        self.buckets = [Bucket(cfg, problems[k:k + per], device=device,
                               stream=torch.cuda.Stream(device=device))
                        for k in range(0, len(problems), per)]
        self.scenarios = [sc for b in self.buckets for sc in b.scenarios]

    def step(self, dts, shared: bool = True, part: int = 2):
        if len(dts) != len(self.scenarios):
            raise ValueError("one dt per scenario")
        k = 0
        for b in self.buckets:
            n = len(b.scenarios)
            b.step(list(dts[k:k + n]), shared, part)
            k += n

    def close(self):
        for b in self.buckets:
            b.close()
        self.buckets, self.scenarios = [], []


def scenario_from_problem(prob, precision: Optional[str] = None, stream=None,
                          **cfg_over) -> Scenario:
    """Build a Scenario from an inputs.Problem (on the given torch stream,
    default the current one)."""
    cfg = config(dim=prob.dim, n_elem=prob.n_elem, degree=prob.degree, width=prob.width,
                 hidden=prob.hidden, precision=precision or prob.precision, **cfg_over)
    return Scenario(cfg, prob.log_perm, prob.porosity, prob.wells, prob.theta0, prob.s0_coefs,
                    stream=stream)
