"""Host-side checks of the C ABI: the library loads, exports every function
include/*.h declares, and its host logic (validation, workspace plan, error
strings, device detection) behaves without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b((?:mg|dg)_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def mg():
    from paper_1904_08684_amd import mg as _mg
    return _mg


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("mg_setup", "mg_vcycle", "mg_solve", "mg_workspace_bytes", "mg_destroy",
                 "mg_set_rhs", "mg_get_solution", "mg_strerror", "mg_last_error"):
        assert want in names
    for want in ("dg_reference_size", "dg_reference_integrals", "dg_volume_integrals", "dg_product_size",
                 "dg_product_integrals", "dg_velocity_projection", "dg_edge_table_size",
                 "dg_edge_integrals", "dg_edge_terms", "dg_rhs", "dg_ssp_rk3_step", "dg_basis_values",
                 "dg_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol(mg):
    missing = [n for n in declared_functions() if not hasattr(mg.lib, n)]
    assert not missing, missing


def test_version_and_strerror(mg):
    assert b"gfx950" in mg.mg_version()
    assert mg.mg_strerror(mg.MG_ENOTCONV) == b"not converged within max_cycles"
    assert mg.mg_strerror(12345) == b"unknown error"


def test_default_opts(mg):
    o = mg.mg_opts()
    mg.mg_default_opts(C.byref(o))
    assert (o.smoother, o.nu1, o.nu2, o.precision, o.max_cycles) == (mg.MG_RBGS, 2, 2, mg.MG_FP64, 100)
    assert abs(o.omega - 0.8) < 1e-15


@pytest.mark.parametrize("dim,n,cent,ok", [
    (2, 129, 0, True), (3, 513, 0, True), (3, 65, 0, True), (2, 5, 0, True),
    (3, 256, 1, True), (2, 64, 1, True), (3, 4, 1, True),
    (2, 128, 0, False),   # not 4 * 2^L + 1
    (3, 100, 0, False),
    (3, 257, 1, False),   # odd cell count
    (4, 9, 0, False),
])
def test_validation(mg, dim, n, cent, ok):
    g = mg.make_grid(min(dim, 3) if dim != 4 else 3, n, cent)
    if dim == 4:
        g.dim = 4
    o = mg.make_opts()
    b = C.c_size_t()
    rc = mg.mg_workspace_bytes(C.byref(g), None, C.byref(o), C.byref(b))
    assert (rc == mg.MG_OK) == ok
    if ok:
        assert b.value > 0 and b.value % 256 == 0


def test_varcoef_needs_cells_and_k(mg):
    g = mg.make_grid(3, 65, mg.MG_NODE)
    o = mg.make_opts()
    st = mg.mg_stencil()
    st.kind = mg.MG_VARCOEF
    b = C.c_size_t()
    assert mg.mg_workspace_bytes(C.byref(g), C.byref(st), C.byref(o), C.byref(b)) == mg.MG_EINVAL
    g = mg.make_grid(3, 64, mg.MG_CELL)
    assert mg.mg_workspace_bytes(C.byref(g), C.byref(st), C.byref(o), C.byref(b)) == mg.MG_EINVAL


def test_bad_options_rejected(mg):
    g = mg.make_grid(2, 129)
    b = C.c_size_t()
    for kw in ({"nu1": 0, "nu2": 0}, {"omega": 0.0}, {"omega": 2.5}, {"max_cycles": 0},
               {"smoother": 7}, {"precision": 3}, {"post_order": 2}, {"cycle": 3}, {"krylov": 2},
               {"krylov": 1, "precision": 1}):
        o = mg.make_opts(**kw)
        assert mg.mg_workspace_bytes(C.byref(g), None, C.byref(o), C.byref(b)) == mg.MG_EINVAL, kw


def test_workspace_scales_with_problem(mg):
    o64 = mg.make_opts(precision=mg.MG_FP64)
    omx = mg.make_opts(precision=mg.MG_MIXED)
    b64 = mg.workspace_bytes(mg.make_grid(3, 513), o64)
    bmx = mg.workspace_bytes(mg.make_grid(3, 513), omx)
    n = 513 ** 3
    # FP64: u, f, r on ~8/7 of the finest size + staging; mixed adds FP32 fields
    assert 4 * 8 * n < b64 < 6 * 8 * n
    assert b64 < bmx < b64 + 3 * 4 * n * 1.3
    # the Krylov vectors add five finest-level FP64 fields
    bk = mg.workspace_bytes(mg.make_grid(3, 513), mg.make_opts(precision=mg.MG_FP64, krylov=1))
    assert 5 * 8 * n < bk - b64 < 5 * 8 * n * 1.1
    # Jacobi adds a double buffer
    bj = mg.workspace_bytes(mg.make_grid(2, 129), mg.make_opts(smoother=mg.MG_JACOBI))
    br = mg.workspace_bytes(mg.make_grid(2, 129), mg.make_opts(smoother=mg.MG_RBGS))
    assert bj > br


def test_setup_without_device_reports_device_error(mg):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    g = mg.make_grid(2, 17)
    o = mg.make_opts()
    h = C.c_void_p()
    rc = mg.mg_setup(C.byref(g), None, None, C.byref(o), C.c_void_p(256), 1 << 30, None, C.byref(h))
    assert rc == mg.MG_EDEVICE
    assert b"device" in mg.mg_last_error(None)


def test_null_safety(mg):
    mg.mg_destroy(None)
    assert mg.mg_vcycle(None, 1) == mg.MG_EINVAL
    assert mg.mg_solve(None, 1e-10, None, None) == mg.MG_EINVAL
    assert mg.mg_pcg(None, 1e-10, 10, None, None) == mg.MG_EINVAL
    assert mg.mg_set_rhs(None, None, 0) == mg.MG_EINVAL


def test_neumann_combinations_rejected_before_any_device_work(mg):
    """Zero-flux walls need a cell grid, FP64 and no Krylov vectors; unknown
    boundary kinds are refused (all checked before the device is touched)."""
    h = C.c_void_p()
    cases = [(mg.make_grid(3, 33, mg.MG_NODE), mg.make_opts(), mg.MG_NEUMANN0),
             (mg.make_grid(3, 32, mg.MG_CELL), mg.make_opts(precision=mg.MG_MIXED), mg.MG_NEUMANN0),
             (mg.make_grid(3, 32, mg.MG_CELL), mg.make_opts(krylov=1), mg.MG_NEUMANN0),
             (mg.make_grid(3, 32, mg.MG_CELL), mg.make_opts(), 7)]
    for g, o, kind in cases:
        bc = mg.mg_bc(kind)
        rc = mg.mg_setup(C.byref(g), None, C.byref(bc), C.byref(o), C.c_void_p(256), 1 << 30, None, C.byref(h))
        assert rc == mg.MG_EINVAL
        assert mg.mg_last_error(None)


def test_galerkin_option_validation(mg):
    """Galerkin coarse operators: node grids, damped Jacobi, FP64 only."""
    b = C.c_size_t()
    ok = mg.make_opts(smoother=mg.MG_JACOBI, coarse_op=mg.MG_COARSE_GALERKIN)
    assert mg.mg_workspace_bytes(C.byref(mg.make_grid(3, 65)), None, C.byref(ok), C.byref(b)) == mg.MG_OK
    for g, kw in ((mg.make_grid(3, 65), {"smoother": mg.MG_RBGS}),
                  (mg.make_grid(3, 65), {"smoother": mg.MG_JACOBI, "precision": mg.MG_MIXED}),
                  (mg.make_grid(3, 64, mg.MG_CELL), {"smoother": mg.MG_JACOBI}),
                  (mg.make_grid(3, 65), {"smoother": mg.MG_JACOBI, "coarse_op": 2})):
        o = mg.make_opts(**{"coarse_op": mg.MG_COARSE_GALERKIN, **kw})
        assert mg.mg_workspace_bytes(C.byref(g), None, C.byref(o), C.byref(b)) == mg.MG_EINVAL, kw


def test_noalloc_rk_step_refuses_sizes_beyond_its_array(mg):
    """dg_ssp_rk3_step_noalloc checks 6 K ne against its fixed 2^23-double
    device array before touching any argument or the device."""
    for k, K in ((0, 1), (1, 3), (3, 10)):
        ne = (1 << 23) // (6 * K) + 1
        code = mg.dg_ssp_rk3_step_noalloc(k, ne, None, None, None, None, None, None, 0, None, None, 9.81, 0.0, 0.0,
                                          None, None, None, None, 1.0, None)
        assert code == mg.MG_EINVAL
        assert b"exceed the fixed scratch" in mg.dg_last_error()
    code = mg.dg_ssp_rk3_step_noalloc(3, 1000, None, None, None, None, None, None, 0, None, None, 9.81, 0.0, 0.0,
                                      None, None, None, None, 1.0, None)
    assert code == mg.MG_EINVAL and mg.dg_last_error() == b""
