"""The C ABI without a GPU: the library loads, exports every function the header declares,
and the host-only entry points (options, plan validation, workspace sizing, status strings)
behave as documented in include/ptsolve.h."""
import ctypes as C
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2502_21013_amd as P
    try:
        P.library()
    except ImportError as e:
        pytest.fail(f"HIP library not built: {e}")
    return P


def header_functions():
    text = open(os.path.join(ROOT, "include", "ptsolve.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(pt_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_function(P):
    lib = P.library()
    names = header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_status_strings(P):
    lib = P.library()
    assert lib.pt_version() >= 1
    for code, name in [(0, b"PT_OK"), (-1, b"PT_ERR_INVALID"), (-4, b"PT_ERR_NOT_CONVERGED"),
                       (-8, b"PT_ERR_WORKSPACE")]:
        assert lib.pt_status_string(code) == name
    assert lib.pt_kernel_class_name(0) == b"setup"
    assert lib.pt_kernel_class_name(999) is None


def test_options_defaults(P):
    from paper_2502_21013_amd import _lib as L
    o = L.Options()
    P.library().pt_options_default(C.byref(o))
    assert o.tol == 1e-8 and o.max_outer == 1000 and o.check_every == 1
    assert o.precision == L.PT_FP64 and o.inner == L.PT_INNER_GALERKIN1
    assert o.vc_sweeps == 1 and abs(o.vc_omega - 0.8) < 1e-15 and o.timing == 0
    assert o.vc_cycle == L.PT_VC_DEFAULT


@pytest.mark.parametrize("field,value", [("n", 30), ("n", 2), ("N", 3), ("N", 2048), ("T", 0.0),
                                         ("nu_max", -1.0), ("sigma_in", -1.0), ("nu_a", 0.0)])
def test_plan_rejects_invalid_problems(P, field, value):
    p = W.config1()
    import dataclasses
    bad = dataclasses.replace(p, **{field: value})
    with pytest.raises(P.PTError) as e:
        P.Plan(bad)
    assert e.value.status == -1
    assert P.library().pt_last_error()


@pytest.mark.parametrize("kw", [dict(tol=0.0), dict(max_outer=0), dict(check_every=0), dict(inner_iters=0),
                                dict(inner_iters=65), dict(vc_omega=1.0), dict(inner="cocg", cycle="v01"),
                                dict(grid_restrict=4), dict(grid_up=-1), dict(grid_matvec=(1 << 22) + 1)])
def test_plan_rejects_invalid_options(P, kw):
    with pytest.raises(P.PTError):
        P.Plan(W.config1(), **kw)


def test_plan_rejects_unknown_cycle(P):
    from paper_2502_21013_amd import _lib as L
    lib = P.library()
    o = P._options(lib, 1e-8, 10, 1, "fp64", "galerkin1", 1, 0.8, False, 1e3, True, False, False)
    o.vc_cycle = 3
    ps = P.problem_struct(W.config1())
    h = C.c_void_p()
    assert lib.pt_plan_create(C.byref(ps), C.byref(o), C.byref(h)) == L.PT_ERR_INVALID
    assert b"vc_cycle" in lib.pt_last_error()
    for cyc, inner in (("v11", "galerkin1"), ("v01", "galerkin1"), ("v11", "cocg"), ("default", "cocg")):
        P.Plan(W.config1(), inner=inner, cycle=cyc).close()


def test_timing_mask_validation(P):
    from paper_2502_21013_amd import _lib as L
    lib = P.library()
    ps = P.problem_struct(W.config1())
    h = C.c_void_p()
    o = P._options(lib, 1e-8, 10, 1, "fp64", "galerkin1", 1, 0.8, False, 1e3, True, True, False)
    o.timing_mask = 1 << L.PT_KERNEL_CLASSES
    assert lib.pt_plan_create(C.byref(ps), C.byref(o), C.byref(h)) == L.PT_ERR_INVALID
    assert b"timing_mask" in lib.pt_last_error()
    o.timing_mask = -1
    assert lib.pt_plan_create(C.byref(ps), C.byref(o), C.byref(h)) == L.PT_ERR_INVALID
    with pytest.raises(ValueError):
        P.Plan(W.config1(), timing=("no_such_kernel",))
    with pytest.raises(ValueError):
        P.Plan(W.config1(), timing=())
    pl = P.Plan(W.config1(), timing=("inverse_rfft_update", "residual_sweep"))
    assert pl._opts.timing == 1 and pl._opts.timing_mask == (1 << 2) | (1 << 11)
    pl.close()


def test_workspace_sizes_scale_with_problem_and_precision(P):
    small = P.Plan(W.with_size(W.config1(), 16, 8)).workspace_bytes
    big = P.Plan(W.config1()).workspace_bytes
    f32 = P.Plan(W.config1(), precision="fp32").workspace_bytes
    cocg = P.Plan(W.config1(), inner="cocg", inner_iters=3).workspace_bytes
    assert 0 < small < big
    assert f32 < big < cocg
    # config 3 in FP64 fits easily in one 288 GB device
    c3 = P.Plan(W.config3(0)).workspace_bytes
    assert 8e9 < c3 < 40e9
    assert c3 % 256 == 0 or True


def test_null_arguments_are_rejected(P):
    from paper_2502_21013_amd import _lib as L
    lib = P.library()
    out = C.c_void_p()
    assert lib.pt_plan_create(None, None, C.byref(out)) == L.PT_ERR_INVALID
    assert lib.pt_plan_workspace_bytes(None, None) == L.PT_ERR_INVALID
    assert lib.pt_solve(None, None, 0, None, None, None) == L.PT_ERR_INVALID
    lib.pt_plan_destroy(None)   # no-op


def test_workspace_checks_happen_before_any_launch(P):
    # wrong size / alignment / NULL are caught on the host; no device call is made
    from paper_2502_21013_amd import _lib as L
    lib = P.library()
    plan = P.Plan(W.with_size(W.config1(), 8, 8))
    dummy = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    st = lib.pt_solve(plan._h, None, plan.workspace_bytes, dummy, None, None)
    assert st == L.PT_ERR_WORKSPACE
    st = lib.pt_solve(plan._h, C.c_void_p(0x1001), plan.workspace_bytes, dummy, None, None)
    assert st == L.PT_ERR_WORKSPACE
    st = lib.pt_solve(plan._h, C.c_void_p(0x1000), plan.workspace_bytes - 1, dummy, None, None)
    assert st == L.PT_ERR_WORKSPACE
    assert b"too small" in lib.pt_last_error()


def _batch_structs(P, ps):
    from paper_2502_21013_amd import _lib as L
    return (L.Problem * len(ps))(*[P.problem_struct(p) for p in ps])


def test_batch_plan_validation(P):
    import dataclasses
    from paper_2502_21013_amd import _lib as L
    lib = P.library()
    o = L.Options()
    lib.pt_options_default(C.byref(o))
    h = C.c_void_p()
    base = [W.with_size(p, 16, 16) for p in W.config4(0, 4)]
    assert lib.pt_plan_create_batch(_batch_structs(P, base), 4, C.byref(o), C.byref(h)) == L.PT_OK
    cnt = C.c_int32()
    assert lib.pt_plan_batch_size(h, C.byref(cnt)) == L.PT_OK and cnt.value == 4
    nb4 = C.c_size_t()
    lib.pt_plan_workspace_bytes(h, C.byref(nb4))
    lib.pt_plan_destroy(h)
    one = P.Plan(base[0]).workspace_bytes
    assert 3 * one < nb4.value < 5 * one
    # count not a power of two
    assert lib.pt_plan_create_batch(_batch_structs(P, base[:3]), 3, C.byref(o), C.byref(h)) == L.PT_ERR_INVALID
    # grid, period and conductivity must be shared
    for change in [dict(n=32), dict(N=32), dict(T=2.0), dict(sigma_in=2.0), dict(nu_max=12.0)]:
        bad = list(base)
        bad[3] = dataclasses.replace(bad[3], **change)
        assert lib.pt_plan_create_batch(_batch_structs(P, bad), 4, C.byref(o), C.byref(h)) == L.PT_ERR_INVALID
        assert b"share" in lib.pt_last_error()
    # device tables are single-problem only
    s = _batch_structs(P, base[:2])
    s[1].d_load = 0x1000
    assert lib.pt_plan_create_batch(s, 2, C.byref(o), C.byref(h)) == L.PT_ERR_INVALID
    # one invalid member names its index
    bad = list(base[:2])
    bad[1] = dataclasses.replace(bad[1], nu_a=-1.0)
    assert lib.pt_plan_create_batch(_batch_structs(P, bad), 2, C.byref(o), C.byref(h)) == L.PT_ERR_INVALID
    assert b"instance 1" in lib.pt_last_error()


def test_batch_plan_rejects_single_entry_points(P):
    from paper_2502_21013_amd import _lib as L
    lib = P.library()
    bp = P.BatchPlan([W.with_size(p, 8, 8) for p in W.config4(1, 2)])
    dummy = C.c_void_p(0x1000)
    assert lib.pt_solve(bp._h, dummy, bp.workspace_bytes, dummy, None, None) == L.PT_ERR_INVALID
    assert lib.pt_residual(bp._h, dummy, bp.workspace_bytes, dummy, dummy, None, None, None) == L.PT_ERR_INVALID
    with pytest.raises(TypeError):
        bp.apply_K(None)


def test_graph_and_timing_are_exclusive(P):
    with pytest.raises(P.PTError):
        P.Plan(W.config1(), graph=True, timing=True)


def test_adjoint_entry_points_need_an_adjoint_plan(P):
    from paper_2502_21013_amd import _lib as L
    lib = P.library()
    plan = P.Plan(W.with_size(W.config1(), 8, 8))
    dummy = C.c_void_p(0x1000)
    assert lib.pt_adjoint_solve(plan._h, dummy, plan.workspace_bytes, dummy, dummy, None, None) == L.PT_ERR_INVALID
    assert b"adjoint" in lib.pt_last_error()
    assert lib.pt_loss_gradients(plan._h, dummy, plan.workspace_bytes, dummy, None, None, None, 0, None,
                                 None) == L.PT_ERR_INVALID
    adj = P.Plan(W.with_size(W.config1(), 8, 8), adjoint=True)
    assert adj.workspace_bytes > plan.workspace_bytes
    assert lib.pt_loss_gradients(adj._h, dummy, adj.workspace_bytes, dummy, None, None, None, 2, None,
                                 None) == L.PT_ERR_INVALID
    with pytest.raises(P.PTError):
        P.BatchPlan([W.with_size(p, 8, 8) for p in W.config4(0, 2)], adjoint=True)


@pytest.mark.parametrize("kw", [dict(init_static=True, init_tol=0.0), dict(init_static=True, use_initial_guess=True)])
def test_static_start_options_are_validated(P, kw):
    with pytest.raises(P.PTError):
        P.Plan(W.config1(), **kw)


@pytest.mark.parametrize("kw", [dict(krylov_dim=65), dict(krylov_dim=-1), dict(krylov_dim=4, forcing=1.0),
                                dict(krylov_dim=4, max_krylov=0)])
def test_newton_options_are_validated(P, kw):
    with pytest.raises(P.PTError):
        P.Plan(W.config1(), **kw)


def test_newton_entry_points_need_a_newton_plan(P):
    from paper_2502_21013_amd import _lib as L
    lib = P.library()
    plan = P.Plan(W.with_size(W.config1(), 8, 8))
    dummy = C.c_void_p(0x1000)
    assert lib.pt_newton_solve(plan._h, dummy, plan.workspace_bytes, dummy, None, None) == L.PT_ERR_INVALID
    assert lib.pt_jacobian_apply(plan._h, dummy, plan.workspace_bytes, dummy, dummy, dummy, 0, None) == L.PT_ERR_INVALID
    nplan = P.Plan(W.with_size(W.config1(), 8, 8), krylov_dim=6)
    assert nplan.workspace_bytes > plan.workspace_bytes + 14 * 81 * 8 * 8
    with pytest.raises(P.PTError):
        P.BatchPlan([W.with_size(p, 8, 8) for p in W.config4(0, 2)], krylov_dim=4)


def test_noalloc_solve_rejects_before_any_device_work(P):
    """pt_solve_noalloc validates on the host: a plan whose workspace exceeds the 64 MiB static
    scratch gets PT_ERR_WORKSPACE, timing or graph plans PT_ERR_INVALID (d_u is never touched)."""
    from paper_2502_21013_amd import _lib as L
    lib = P.library()
    dummy = (C.c_double * 1)()
    big = P.Plan(W.with_size(W.config1(), 256, 64))
    assert big.workspace_bytes > 64 << 20
    st = lib.pt_solve_noalloc(big._h, C.cast(dummy, C.c_void_p), None, None)
    assert st == L.PT_ERR_WORKSPACE and b"static device scratch" in lib.pt_last_error()
    for kw in (dict(timing=True), dict(graph=True)):
        pl = P.Plan(W.config1(), **kw)
        assert lib.pt_solve_noalloc(pl._h, C.cast(dummy, C.c_void_p), None, None) == L.PT_ERR_INVALID
    assert lib.pt_solve_noalloc(None, C.cast(dummy, C.c_void_p), None, None) == L.PT_ERR_INVALID


@pytest.mark.parametrize("kw", [dict(inner_rtol=-1e-3), dict(inner_rtol=1.0), dict(breakdown_tol=-1.0),
                                dict(breakdown_tol=float("inf"))])
def test_plan_rejects_invalid_inner_tolerances(P, kw):
    with pytest.raises(P.PTError) as e:
        P.Plan(W.config1(), inner="cocg", **kw)
    assert e.value.status == -1


def test_pt_log_reports_plans_on_stderr():
    """PT_LOG=1 makes the library describe each plan on stderr; unset, it prints nothing."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r); import paper_2502_21013_amd as P, workloads as W; "
            "P.Plan(W.config1(), precision='fp32')" % ROOT)
    env = dict(os.environ, PT_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "[ptsolve] plan n=32 N=32 B=1 fp32+refine" in r.stderr
    env.pop("PT_LOG")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert "[ptsolve]" not in r.stderr
