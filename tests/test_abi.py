"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function that include/schwinger_hmc.h declares, and validates its arguments on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "schwinger_hmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hmc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1512_03812_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libschwinger_hmc.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_paper_operations():
    names = declared_functions()
    for required in ["hmc_init", "hmc_dslash", "hmc_dslash_dagger", "hmc_cg_solve",
                     "hmc_fermion_force", "hmc_gauge_force", "hmc_update_links",
                     "hmc_update_momenta", "hmc_fg_shifted_force", "hmc_trajectory"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_1512_03812_amd import _lib
    assert set(_lib.exported_symbols()) == set(declared_functions())


def test_init_validates_arguments(lib):
    ctx = ctypes.c_void_p()
    assert lib.hmc_init(ctypes.byref(ctx), 7, 2.0, 0.1, 1) == -1   # odd L
    assert lib.hmc_init(ctypes.byref(ctx), 0, 2.0, 0.1, 1) == -1
    assert lib.hmc_init(ctypes.byref(ctx), 8, float("nan"), 0.1, 1) == -1
    assert lib.hmc_init(ctypes.byref(ctx), 8, 2.0, float("inf"), 1) == -1
    assert lib.hmc_init(None, 8, 2.0, 0.1, 1) == -1
    assert lib.hmc_init_ex(ctypes.byref(ctx), 8, 6, 2.0, 0.1, 1) == 0
    assert lib.hmc_destroy(ctx) == 0


def test_workspace_size_and_geometry(lib):
    ctx = ctypes.c_void_p()
    Lx = (ctypes.c_int * 3)(16, 8, 4)
    Lt = (ctypes.c_int * 3)(16, 6, 2)
    beta = (ctypes.c_double * 3)(1.0, 2.0, 3.0)
    m0 = (ctypes.c_double * 3)(0.1, 0.2, 0.05)
    assert lib.hmc_batch_init(ctypes.byref(ctx), 3, Lx, Lt, beta, m0, 5) == 0
    n = ctypes.c_int()
    vt = ctypes.c_longlong()
    offs = (ctypes.c_int * 3)()
    assert lib.hmc_geometry(ctx, ctypes.byref(n), ctypes.byref(vt), offs, None, None) == 0
    assert n.value == 3 and vt.value == 256 + 48 + 8
    assert list(offs) == [0, 256, 304]
    # at least: 9 real link fields, 13 FP64 spinors, two complex link fields, the FP32 link
    # angles and 7 FP32 solver spinors
    assert lib.hmc_workspace_bytes(ctx) >= vt.value * (9 * 16 + 13 * 32 + 2 * 32 + 8 + 7 * 16)
    assert lib.hmc_destroy(ctx) == 0


def test_unbound_context_is_rejected_without_touching_the_gpu(lib):
    ctx = ctypes.c_void_p()
    assert lib.hmc_init(ctypes.byref(ctx), 8, 2.0, 0.1, 1) == 0
    buf = ctypes.create_string_buffer(64)
    assert lib.hmc_dslash(ctx, buf, buf) == -1
    assert lib.hmc_trajectory(ctx, 4, 1.0, 4, 2, 0, None) == -1
    assert b"workspace" in lib.hmc_last_error(ctx)
    assert lib.hmc_set_solver(ctx, -1.0, 10, 0.1) == -1
    assert lib.hmc_set_solver(ctx, 1e-10, 10, 1.5) == -1
    assert lib.hmc_set_solver(ctx, 1e-10, 10, 0.1) == 0
    assert lib.hmc_set_trajectory_counter(ctx, 17) == 0
    assert lib.hmc_get_trajectory_counter(ctx) == 17
    assert lib.hmc_set_fg_mode(ctx, 2) == -1
    assert lib.hmc_set_fg_mode(ctx, 1) == 0 and lib.hmc_set_fg_mode(ctx, 0) == 0
    assert lib.hmc_force_gradient_term(ctx, 2, buf, buf, 0, None) == -1
    assert lib.hmc_hessian_vector(ctx, 0, None, buf, buf, 0, None) == -1
    assert lib.hmc_stream_copy(ctx, buf, buf, 16) == -1
    assert lib.hmc_set_cg_groups(ctx, 0) == -1 and lib.hmc_set_cg_groups(ctx, 5) == -1
    assert lib.hmc_set_cg_groups(ctx, 3) == 0 and lib.hmc_set_cg_groups(ctx, 1) == 0
    assert lib.hmc_set_cg_groups(ctx, 2) == 0 and lib.hmc_set_cg_groups(ctx, 1) == 0
    assert lib.hmc_set_fused_cg(ctx, 1) == 0 and lib.hmc_set_fused_cg(ctx, 0) == 0
    ctxs = (ctypes.c_void_p * 9)(*([ctx.value] * 9))
    assert lib.hmc_trajectories_concurrent(None, 1, 4, 1.0, 4, 2, 0, None, None) == -1
    assert lib.hmc_trajectories_concurrent(ctxs, 0, 4, 1.0, 4, 2, 0, None, None) == -1
    assert lib.hmc_trajectories_concurrent(ctxs, 9, 4, 1.0, 4, 2, 0, None, None) == -1
    assert lib.hmc_trajectories_concurrent(ctxs, 1, 4, 1.0, 4, 2, 0, None, None) == -1  # unbound
    assert lib.hmc_destroy(ctx) == 0
    assert lib.hmc_destroy(None) == -1


def test_bind_rejects_small_or_misaligned_workspace(lib):
    ctx = ctypes.c_void_p()
    assert lib.hmc_init(ctypes.byref(ctx), 8, 2.0, 0.1, 1) == 0
    need = lib.hmc_workspace_bytes(ctx)
    assert lib.hmc_bind(ctx, None, need, None) == -1
    assert lib.hmc_bind(ctx, ctypes.c_void_p(4096 + 8), need, None) == -1    # misaligned
    assert lib.hmc_bind(ctx, ctypes.c_void_p(4096), need - 1, None) == -2   # too small
    assert lib.hmc_destroy(ctx) == 0


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1512_03812_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()
