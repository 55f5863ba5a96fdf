"""The C-ABI library loads and exports every function include/hsdc.h declares;
argument checks fail with HSDC_EINVAL before any device work (no GPU needed)."""
import ctypes

import pytest

from paper_2405_19994_amd import hsdc as H


def test_header_symbols_exported():
    names = H.header_functions()
    assert "hsdc_init_state" in names and "hsdc_pfasst_iter" in names
    lib = H.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layout_matches_header():
    # field order and C types of the two public structs
    assert ctypes.sizeof(H.Problem) == 4 * 4 + 8 + 24 + 8 + 8 + 8 + 24 + 8 + 24 + 8
    assert [f for f, _ in H.Problem._fields_][:5] == ["dim", "nx", "ny", "nz", "dx"]
    assert ctypes.sizeof(H.Stats) == 9 * 8
    # levels, M[2], space_coarsen, P | dt | max_iter | tol | burn_in, solver |
    # cg_rtol | cg_maxit, coarse_fp32 | coarse_cg_rtol | residual_norm (+ padding)
    assert ctypes.sizeof(H.Method) == 88
    assert H.Method.solver.offset == 52
    assert H.Method.coarse_cg_rtol.offset == 72
    assert H.Method.residual_norm.offset == 80
    assert H.Method.prefix_stop.offset == 84


def _init(p, m):
    ptr = ctypes.c_void_p()
    code = H.lib().hsdc_init_state(ctypes.byref(p), ctypes.byref(m), None, None, ctypes.byref(ptr))
    return code, ptr


@pytest.mark.parametrize("bad", [
    dict(dims=(0,)), dict(dx=-1.0), dict(chi=0.0), dict(sigma=(-1.0, 1, 1)),
])
def test_bad_problem_is_einval(bad):
    kw = dict(dims=(16,), dx=0.01)
    kw.update(bad)
    p = H.make_problem(**kw)
    if "dims" in bad:
        p.nx = 0
    code, ptr = _init(p, H.make_method())
    assert code == -1 and not ptr.value
    assert H.lib().hsdc_last_error(None)


@pytest.mark.parametrize("bad", [
    dict(M=(0, 1)), dict(M=(9, 1)), dict(dt=0.0), dict(max_iter=0), dict(cg_rtol=0.0),
    dict(levels=4), dict(levels=1, P=4), dict(levels=3, M=(6, 3, 1), P=2, coarse_fp32=1),
    dict(levels=3, M=(6, 3, 0), P=2), dict(levels=2, M=(4, 2), P=2, prefix_stop=2),
    dict(levels=3, M=(6, 3, 1), P=2, prefix_stop=1), dict(levels=2, M=(4, 2), space_coarsen=2, P=2),
    dict(levels=2, M=(4, 2), P=2, coarse_fp32=2), dict(levels=2, M=(4, 2), P=2, coarse_cg_rtol=1.0),
    dict(solver=4), dict(solver=-1), dict(residual_norm=2),
    dict(levels=2, M=(4, 2), P=2, solver=3, coarse_fp32=1),
])
def test_bad_method_is_einval(bad):
    p = H.make_problem((15,), 0.01)
    code, ptr = _init(p, H.make_method(**bad))
    assert code == -1 and not ptr.value


def test_three_levels_need_meshes_divisible_by_four():
    """Two space coarsenings halve every axis twice: 12 x 6 is rejected."""
    m = H.make_method(M=(6, 3, 1), levels=3, space_coarsen=2, P=2)
    code, ptr = _init(H.make_problem((12, 6), 0.025), m)
    assert code == -1 and not ptr.value
    assert b"divisible by 4" in H.lib().hsdc_last_error(None)


@pytest.mark.parametrize("case", ["order3", "order4_cg", "order4_pernode", "dct_pernode"])
def test_fourth_order_and_dct_arguments_are_checked(case):
    """fd_order is 2 or 4; the fourth-order stencil needs a uniform sigma and
    the DCT-II solver (solver 3), which needs a uniform sigma too."""
    p = H.make_problem((16, 8), 0.025, fd_order=4)
    m = H.make_method(M=4, solver="dct")
    if case == "order3":
        p.fd_order = 3
    elif case == "order4_cg":
        m = H.make_method(M=4)
    else:
        p.sigma_node = 8  # never dereferenced: rejected before any device work
        if case == "dct_pernode":
            p.fd_order = 2
    code, ptr = _init(p, m)
    assert code == -1 and not ptr.value
    assert H.lib().hsdc_last_error(None)


def test_null_context_calls_are_einval():
    L = H.lib()
    assert L.hsdc_advance(None, 1) == -1
    assert L.hsdc_sdc_sweep(None, 0, 0, 1) == -1
    assert L.hsdc_pfasst_iter(None, None, None) == -1
    assert L.hsdc_residual(None, 0, None) == -1
    assert L.hsdc_current_step(None) == -1
    L.hsdc_destroy(None)
    assert L.hsdc_phi(10, None, 0, None, None) == -1
    assert L.hsdc_colloc_coefficients(0, 1, None, None, None, None) == -1


def _batch(probs, m):
    arr = (H.Problem * len(probs))(*probs)
    ptr = ctypes.c_void_p()
    code = H.lib().hsdc_init_batch(arr, len(probs), ctypes.byref(m), None, None, ctypes.byref(ptr))
    return code, ptr


@pytest.mark.parametrize("bad", ["dx", "levels", "count", "sigma"])
def test_bad_batch_is_einval(bad):
    """Tissues of a batch share everything but their mesh, sigma field and
    stimulus weights; the method is serial.  Rejected before any device call."""
    probs = [H.make_problem((12, 10), 0.025), H.make_problem((8, 14), 0.025)]
    m = H.make_method(M=4, max_iter=4)
    if bad == "dx":
        probs[1] = H.make_problem((8, 14), 0.03)
    elif bad == "levels":
        m = H.make_method(M=(4, 2), levels=2, P=2)
    elif bad == "sigma":
        probs[1] = H.make_problem((8, 14), 0.025, sigma=(2.0, 1.0, 1.0))
    if bad == "count":
        ptr = ctypes.c_void_p()
        code = H.lib().hsdc_init_batch(None, 0, ctypes.byref(m), None, None, ctypes.byref(ptr))
    else:
        code, ptr = _batch(probs, m)
    assert code == -1 and not ptr.value
    assert H.lib().hsdc_last_error(None)



def test_noalloc_solve_rejects_large_meshes_before_device_work():
    """The no-allocation solve checks the mesh against HSDC_NOALLOC_MAX_NODES
    before it touches the device (the pointers are never dereferenced)."""
    p = H.make_problem((1024, 513), 0.025)
    code = H.lib().hsdc_diffusion_solve_noalloc(ctypes.byref(p), 0.01, ctypes.c_void_p(8),
                                                ctypes.c_void_p(8), 1e-12, 100, None, None)
    assert code == -1
    assert b"HSDC_NOALLOC_MAX_NODES" in H.lib().hsdc_last_error(None)
    assert H.NOALLOC_MAX_NODES == 524288
