"""The C ABI: the library loads without a GPU, exports every function that
include/srwcr.h declares, and its host-only entry points validate arguments."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "srwcr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?!typedef\b)(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for", "return")))


def test_header_declares_the_bound_functions():
    from paper_1804_05061_amd import _lib
    assert set(header_functions()) == set(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_1804_05061_amd import _lib
    L = _lib.load()
    for name in header_functions():
        assert hasattr(L, name), name


def test_ctrl_dims_and_validation_without_gpu():
    import paper_1804_05061_amd as S
    p = S.Problem((256, 256, 128), (256, 256, 128), 64, (6, 6, 6), (10, 10, 10))
    assert p.ctrl_dims == (29, 29, 16)
    assert S.Problem((64, 64, 64), (64, 64, 64), 32, (4, 4, 4), (8, 8, 8)).ctrl_dims == (11, 11, 11)
    with pytest.raises(S.SrwcrError):
        S.Problem((64, 64, 64), (64, 64, 64), 32, (4, 4, 4), (0, 8, 8)).ctrl_dims
    from paper_1804_05061_amd import _lib
    L = _lib.load()
    assert L.srwcr_plan_create(None, None) == -1
    assert b"NULL" in L.srwcr_last_error()
    opts = _lib.SrwcrLbfgsOpts()
    L.srwcr_lbfgs_default_opts(ctypes.byref(opts))
    assert (opts.levels, list(opts.max_iter), opts.history, opts.stall_window) == (3, [200, 200, 120], 5, 20)


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1804_05061_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.replace("Oracle", "").lower() or f == "build.py", f


def test_new_entry_points_reject_null_arguments_without_gpu():
    """RaPTOR, the fixed-image gradient and the validation of the node-region
    setting fail with SRWCR_E_INVALID_ARG before any device work."""
    import paper_1804_05061_amd as S
    from paper_1804_05061_amd import _lib
    L = _lib.load()
    h = ctypes.c_void_p()
    assert L.raptor_patches_create(None, None, 1, ctypes.byref(h)) == -1
    assert L.raptor_workspace_bytes(None, None) == 0
    assert L.raptor_eval(None, None, None, None, None, 0, None, None, 0, None) == -1
    assert L.raptor_grad(None, None, None, None, None, 0, None, None, None, 0, None) == -1
    assert L.srwcr_grad_fixed(None, None, None, None, 0, None, None, None, 0, None) == -1
    # spatial_bins must be all 0 (regions at the FFD nodes) or all in 4..64
    assert S.Problem((64, 64, 64), (64, 64, 64), 32, (0, 0, 0), (5, 5, 5)).n_regions == 16 ** 3
    p = S.Problem((64, 64, 64), (64, 64, 64), 32, (0, 4, 4), (5, 5, 5))
    assert L.srwcr_plan_create(ctypes.byref(p.c()), ctypes.byref(h)) == -1
    assert b"spatial_bins" in L.srwcr_last_error()


def test_boundary_rejects_bad_arguments_without_gpu():
    """Argument checks that run before any device work: batches outside 1..32
    problems or without plans, profiling without a plan, and the srwcr_grad
    family and the no-alloc entry point without a plan."""
    from paper_1804_05061_amd import _lib
    L = _lib.load()
    h = ctypes.c_void_p()
    plans = (ctypes.c_void_p * 33)()
    assert L.srwcr_batch_create(0, plans, ctypes.byref(h)) == -1
    assert L.srwcr_batch_create(33, plans, ctypes.byref(h)) == -1
    assert b"outside 1..32" in L.srwcr_last_error()
    assert L.srwcr_batch_create(1, None, ctypes.byref(h)) == -1
    assert L.srwcr_batch_create(1, plans, None) == -1
    assert L.srwcr_batch_create(1, plans, ctypes.byref(h)) == -1          # plans[0] is NULL
    assert L.srwcr_batch_workspace_bytes(None) == 0
    assert L.srwcr_grad_batched(None, None, None, 0, None) == -1
    assert L.srwcr_profile(None, 1) == -1
    ms = (ctypes.c_double * 6)()
    assert L.srwcr_profile_read(None, ms, None) == -1
    assert L.srwcr_eval(None, None, None, None, None, None, 0, None) == -1
    assert L.srwcr_grad(None, None, None, None, None, None, None, 0, None) == -1
    assert L.srwcr_grad_dense(None, None, None, None, None, None, None, 0, None) == -1
    assert L.srwcr_grad_noalloc(None, None, None, None, None, None, None) == -1
    assert L.srwcr_workspace_bytes(None) == 0
