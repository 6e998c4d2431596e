"""Host-side checks of the C ABI (no device work): the library loads, exports
every function include/crv.h declares, validates configurations and sizes its
workspace consistently."""
import os
import re

import pytest

from paper_2604_20731_amd import crv, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "crv.h")).read()
    return sorted(set(re.findall(r"\b(crv_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert "crv_init" in names and "crv_step" in names
    for n in names:
        assert hasattr(crv.LIB, n), n
    assert sorted(crv.EXPORTED) == names


@pytest.mark.parametrize("dim,width,hidden", [(2, 32, 3), (2, 64, 4), (2, 128, 4), (3, 128, 4)])
def test_param_count_matches_layout(dim, width, hidden):
    cfg = crv.config(dim=dim, width=width, hidden=hidden)
    assert crv.param_count(cfg) == inputs.n_params(dim, width, hidden)
    assert crv.param_count(cfg) == inputs.theta_xavier(dim, width, hidden, 0).size


def test_config_validation_errors():
    bad = [dict(dim=4), dict(n_elem=2), dict(degree=5), dict(width=48), dict(hidden=0),
           dict(mu_g=0.0), dict(lr=-1.0), dict(well_radius=0.0), dict(substeps=0),
           dict(precision=7), dict(dim=3, n_elem=300),
           dict(dim=3, width=64, hidden=3, precision="bf16")]
    for kw in bad:
        cfg = crv.config(**kw)
        with pytest.raises(crv.CrvError) as ei:
            crv.workspace_size(cfg)
        assert ei.value.status == crv.CRV_EINVAL, kw


def test_workspace_grows_with_grid_and_precision():
    a = crv.workspace_size(crv.config(n_elem=64, width=64, hidden=4))
    b = crv.workspace_size(crv.config(n_elem=128, width=64, hidden=4))
    c = crv.workspace_size(crv.config(n_elem=128, width=64, hidden=4, precision="fp64"))
    assert 0 < a < b < c
    assert a % 256 == 0


def test_workspace_3d():
    """3D interior arrays are padded to mp^3 and the Gram lines to m*mp."""
    w2 = crv.workspace_size(crv.config(dim=2, n_elem=128, width=128, hidden=4, precision="bf16"))
    w3 = crv.workspace_size(crv.config(dim=3, n_elem=128, width=128, hidden=4, precision="bf16"))
    assert w3 > w2
    # nodal, coefficient and interior arrays alone
    assert w3 > 4 * (10 * 129 ** 3 + 3 * 130 ** 3 + 5 * 128 ** 3)


def test_defaults():
    cfg = crv.config()
    assert cfg.lr == 1e-4 and cfg.adam_iters == 100 and cfg.substeps == 10
    assert cfg.mu_w == 1.0 and cfg.mu_g == 0.1 and cfg.relperm_exp == 2.0


def test_batch_and_state_argument_errors():
    """Argument checks that run before any device work (no GPU needed)."""
    import ctypes as C
    assert crv.LIB.crv_step_batch(None, None, -1) == crv.CRV_EINVAL
    assert crv.LIB.crv_step_batch(None, None, 1) == crv.CRV_EINVAL
    ctxs = (C.c_void_p * 1)(None)
    dts = (C.c_double * 1)(1e-3)
    assert crv.LIB.crv_step_batch(ctxs, dts, 1) == crv.CRV_EINVAL
    assert crv.LIB.crv_step_batch(None, None, 0) == crv.CRV_OK
    assert crv.LIB.crv_set_log_perm(None, None) == crv.CRV_EINVAL
    assert crv.LIB.crv_last_error().decode()  # a message accompanies every error


def test_precision_names_cover_the_enum():
    import re
    text = open(os.path.join(ROOT, "include", "crv.h")).read()
    enum = dict((k, int(v)) for k, v in re.findall(r"CRV_PREC_(\w+)\s*=\s*(\d+)", text))
    assert sorted(enum.values()) == sorted(crv.PREC.values())
    for name in ("fp32", "bf16", "fp64", "bf16x3", "bf16x3f"):
        cfg = crv.config(width=64, hidden=4, precision=name)
        assert crv.workspace_size(cfg) > 0


def test_gravity_config_and_galerkin_argument_errors():
    """Gravity fields sit at the end of crv_config (the binding's structure
    matches the header's order), default to zero and are validated; the
    direct-solver entry points reject a missing context before any device
    work."""
    import ctypes as C
    cfg = crv.config()
    assert cfg.gravity == 0.0 and cfg.rho_w == 0.0 and cfg.rho_g == 0.0
    names = [f for f, _ in crv.CrvConfig._fields_]
    assert names[-4:] == ["gravity", "rho_w", "rho_g", "boundary_factor"]
    assert crv.workspace_size(crv.config(gravity=9.81, rho_w=1.0, rho_g=0.5)) > 0
    for bad in (dict(gravity=-1.0), dict(rho_w=-0.1), dict(rho_g=float("nan"))):
        n = C.c_size_t()
        c = crv.config(**bad)
        assert crv.LIB.crv_workspace_size(C.byref(c), C.byref(n)) == crv.CRV_EINVAL, bad
    it, rr = C.c_int(), C.c_double()
    assert crv.LIB.crv_pressure_galerkin(None, 10, 1e-6, 1, None, C.byref(it),
                                         C.byref(rr)) == crv.CRV_EINVAL
    assert crv.LIB.crv_step_galerkin(None, 1e-3, 10, 1e-6, 1, None, None) == crv.CRV_EINVAL
    assert "context" in crv.LIB.crv_last_error().decode()


def test_precond_constants_match_the_header():
    """The binding's preconditioner codes are the header's CRV_PRECOND_*."""
    import re
    from pathlib import Path
    text = (Path(__file__).resolve().parents[1] / "include" / "crv.h").read_text()
    found = {m.group(1).lower(): int(m.group(2))
             for m in re.finditer(r"#define CRV_PRECOND_(\w+) (\d+)", text)}
    assert found == crv.PRECOND


def test_config_struct_matches_header():
    """The binding's crv_config has the header's fields, in order, with the
    header's C types (read from the struct declaration in include/crv.h)."""
    import ctypes as C
    import re
    from pathlib import Path
    text = (Path(__file__).resolve().parents[1] / "include" / "crv.h").read_text()
    body = re.search(r"typedef struct \{(.*?)\} crv_config;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    header = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, rest = decl.split(None, 1)
        header += [(n.strip(), ctype) for n in rest.split(",")]
    ctypes_of = {"int": C.c_int, "double": C.c_double}
    assert [(n, ctypes_of[t]) for n, t in header] == list(crv.CrvConfig._fields_)
    assert crv.config().boundary_factor == 0
    n = C.c_size_t()
    assert crv.LIB.crv_workspace_size(C.byref(crv.config(boundary_factor=2)), C.byref(n)) == -1
    assert crv.workspace_size(crv.config(boundary_factor=1)) > 0


def test_splitmix64_published_vector():
    """The tests' SplitMix64 (the generator of the library's seeded default
    parameters) reproduces the published outputs for seed 1234567."""
    from helpers import splitmix64
    assert [splitmix64(1234567, k) for k in range(5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]
