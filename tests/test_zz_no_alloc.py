"""The allocation-free FP64 solve (hmc_cg_solve_noalloc, scratch in the library's static
device array) against hmc_cg_solve on the same contexts, through the C ABI: two calls in a row,
the second on a smaller context, each bit for bit equal to the workspace-scratch solve; sizes
beyond the static array's limits are refused with an error."""
import ctypes

import numpy as np
import pytest

from tests import inputs
from tests.gpu_helpers import Batch, hmc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solve_both(shapes, seed, tol=1e-12, max_iter=100000):
    b = Batch(shapes, seed=seed)
    b.set_q([inputs.random_angles(s[0], s[1], seed + i) for i, s in enumerate(shapes)])
    phi = b.spinor_to_native([inputs.random_spinor(s[0], s[1], seed + 50 + i)
                              for i, s in enumerate(shapes)])
    lib, ctx = b.lat._lib, b.lat._ctx
    n = len(shapes)
    x_ref = b.lat.new_spinor()
    x_new = b.lat.new_spinor().fill_(7.0)
    i_ref = (hmc()._lib.CGInfo * n)()
    i_new = (hmc()._lib.CGInfo * n)()
    rc_ref = lib.hmc_cg_solve(ctx, ctypes.c_void_p(phi.data_ptr()), ctypes.c_void_p(x_ref.data_ptr()),
                              tol, max_iter, 0, i_ref)
    rc_new = lib.hmc_cg_solve_noalloc(ctx, ctypes.c_void_p(phi.data_ptr()),
                                      ctypes.c_void_p(x_new.data_ptr()), tol, max_iter, i_new)
    torch.cuda.synchronize()
    return b, rc_ref, rc_new, x_ref, x_new, i_ref, i_new


def _same(i_ref, i_new, n):
    for k in range(n):
        a, b = i_ref[k], i_new[k]
        assert (a.iters, a.converged, a.reliable_updates) == (b.iters, b.converged, b.reliable_updates)
        assert a.rel_resid == b.rel_resid and a.rel_resid_true == b.rel_resid_true


def test_noalloc_solve_matches_workspace_solve_twice_with_a_smaller_second_input():
    big = [(16, 16, 2.0, 0.1), (32, 32, 3.0, 0.05), (8, 8, 1.0, 0.2), (44, 46, 2.5, 0.1), (2, 2, 2.0, 0.3)]
    b, rc_ref, rc_new, x_ref, x_new, i_ref, i_new = _solve_both(big, 11)
    assert rc_ref == 0 and rc_new == 0
    assert torch.equal(x_ref, x_new)
    _same(i_ref, i_new, len(big))
    assert all(i_new[k].converged for k in range(len(big)))
    small = [(8, 8, 2.0, 0.1), (4, 6, 1.5, 0.3)]
    b2, rc_ref, rc_new, x_ref, x_new, i_ref, i_new = _solve_both(small, 23)
    assert rc_ref == 0 and rc_new == 0
    assert torch.equal(x_ref, x_new)
    _same(i_ref, i_new, len(small))
    # an iteration cap: the same unconverged iterate and HMC_E_NOCONV from both
    b3, rc_ref, rc_new, x_ref, x_new, i_ref, i_new = _solve_both(small, 29, max_iter=3)
    assert rc_ref == rc_new == -3
    assert torch.equal(x_ref, x_new)
    _same(i_ref, i_new, len(small))


def test_noalloc_solve_refuses_sizes_beyond_its_scratch():
    m = hmc()
    # a chain above the persistent solver's 2048 sites
    b = Batch([(64, 64, 2.0, 0.1)])
    out = b.lat.new_spinor()
    with pytest.raises(m.HMCError) as e:
        b.lat.cg_solve_noalloc(b.lat.new_spinor(), out)
    assert e.value.code == -1
    # more sites than the static array holds (33 chains of 2048 sites)
    b = Batch([(32, 64, 2.0, 0.1)] * 33)
    with pytest.raises(m.HMCError) as e:
        b.lat.cg_solve_noalloc(b.lat.new_spinor(), b.lat.new_spinor())
    assert e.value.code == -2
