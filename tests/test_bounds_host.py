"""Host-only bounds check of every plan's launch geometry and workspace layout (no GPU needed):
pt_plan_check_bounds walks each workgroup of each sweeping kernel with the kernels' own range
helpers and checks every index range, partial-sum slot and LDS request against its buffer, for
the configurations of the build and the extremes of the ABI's ranges."""
import ctypes as C
import dataclasses

import pytest

import workloads as W


@pytest.fixture(scope="module")
def P():
    import paper_2502_21013_amd as P
    P.library()
    return P


def check(P, plan):
    msg = C.create_string_buffer(512)
    st = P.library().pt_plan_check_bounds(plan._h, msg, 512)
    assert st == 0, msg.value.decode()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c5"])
def test_config_plans_are_in_bounds(P, name, precision):
    p = {"c1": W.config1(), "c2": W.config2(0), "c3": W.config3(0), "c5": W.config2(0)}[name]
    for kw in (dict(), dict(inner="cocg", inner_iters=3), dict(adjoint=True), dict(krylov_dim=8),
               dict(grid_slot=8, grid_team=8), dict(grid_slot=4194304, grid_team=4194304), dict(xcd_remap=False),
               dict(grid_restrict=16384, grid_up=4096, grid_matvec=4096),
               dict(grid_restrict=8, grid_up=4194304, grid_matvec=8),
               dict(inner="cocg", grid_restrict=2048, grid_up=8, grid_matvec=4194304)):
        check(P, P.Plan(p, precision=precision, **kw))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batching_plans_are_in_bounds(P, precision):
    from paper_2502_21013_amd.batch import plan_groups
    probs = W.config4(0)
    for ix in plan_groups(probs):
        check(P, P.BatchPlan([probs[i] for i in ix], precision=precision))
        check(P, P.BatchPlan([probs[i] for i in ix], precision=precision, inner="cocg", inner_iters=2))


@pytest.mark.parametrize("n,N", [(4, 4), (4, 1024), (8, 2), (64, 1024), (4096, 4), (2048, 64), (4096, 1024)])
def test_extreme_sizes_are_in_bounds(P, n, N):
    if N < 4:
        pytest.skip("N >= 4 by the ABI")
    for precision in ("fp64", "fp32"):
        check(P, P.Plan(W.with_size(W.config1(), n, N), precision=precision))


def test_largest_batch_is_in_bounds(P):
    # 1024 instances of N = 128: 65536 slots per node, the ABI's limit
    probs = [dataclasses.replace(W.with_size(W.config1(), 8, 128), J0=1.0 + k) for k in range(512)]
    check(P, P.BatchPlan(probs, precision="fp32", inner="cocg"))


def _region_plan_status(P, p, **opts):
    """Create a region-mode plan through the ABI with a placeholder device pointer for the region
    table (plan creation and the bounds walk never dereference it); returns (status, plan handle)."""
    from paper_2502_21013_amd import _lib as L
    lib = P.library()
    ps = P.problem_struct(dataclasses.replace(p, regions=None))
    arr = (L.Region * len(p.regions))(*[L.Region(r.sigma, r.a, r.b, r.c, r.d, r.j, r.nu_hat) for r in p.regions])
    ps.law = {"rational": L.PT_NU_RATIONAL, "expcap": L.PT_NU_EXPCAP}[p.law]
    ps.nregions, ps.regions, ps.d_region = len(p.regions), arr, 0x1000
    o = P._options(lib, 1e-8, 100, 1, opts.pop("precision", "fp64"), opts.pop("inner", "galerkin1"), 1, 0.8, False,
                   1e3, True, False, False, **opts)
    h = C.c_void_p()
    st = lib.pt_plan_create(C.byref(ps), C.byref(o), C.byref(h))
    return st, h, arr


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n,grid", [(16, 0), (64, 66), (512, 0)])
def test_region_khat_plans_are_in_bounds(P, precision, n, grid):
    # per-region Khat: the stiffness tables of every level join the workspace layout
    st, h, _ = _region_plan_status(P, W.transformer(n, 8, khat_factor=1.2), precision=precision, grid_slot=grid)
    assert st == 0, P.library().pt_last_error()
    msg = C.create_string_buffer(512)
    assert P.library().pt_plan_check_bounds(h, msg, 512) == 0, msg.value.decode()
    P.library().pt_plan_destroy(h)


def test_region_khat_validation_and_inner_methods(P):
    p = W.transformer(16, 8, khat_factor=1.2)
    for kw in (dict(inner="cocg"), dict(cycle="v11")):
        st, h, _ = _region_plan_status(P, p, **kw)
        assert st == 0, P.library().pt_last_error()
        msg = C.create_string_buffer(512)
        assert P.library().pt_plan_check_bounds(h, msg, 512) == 0, msg.value.decode()
        P.library().pt_plan_destroy(h)
    bad = dataclasses.replace(p, regions=(dataclasses.replace(p.regions[0], nu_hat=-1.0),) + p.regions[1:])
    st, h, _ = _region_plan_status(P, bad)
    assert st == -1 and b"nu_hat" in P.library().pt_last_error()
