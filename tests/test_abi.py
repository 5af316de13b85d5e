"""The C-ABI library loads and exports every symbol include/ctmrg.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ctmrg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctmrg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["ctmrg_init", "ctmrg_step", "ctmrg_run_to_fixed_point", "ctmrg_observables",
                     "ctmrg_backward", "ctmrg_export_state", "ctmrg_import_state", "ctmrg_destroy",
                     "ctmrg_last_error", "ctmrg_workspace_size", "ctmrg_eigh_topk",
                     "ctmrg_fixed_point_derivative"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2004_08669_amd import ctmrg
    if not os.path.exists(ctmrg.LIB_PATH):
        pytest.skip("libctmrg.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(ctmrg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares the same set
    lib2 = ctmrg.load()
    assert lib2 is not None


def test_invalid_arguments_fail_without_a_gpu_call():
    from paper_2004_08669_amd import ctmrg
    if not os.path.exists(ctmrg.LIB_PATH):
        pytest.skip("libctmrg.so not built")
    lib = ctmrg.load()
    # argument validation happens before any device work
    import numpy as np
    V = np.array([[1.0], [-1.0]])
    h = ctypes.c_void_p()
    assert lib.ctmrg_init(1, 1, ctmrg._p(V), 1.0, 4, None, ctypes.byref(h)) == 1   # q < 2
    assert lib.ctmrg_init(2, 1, ctmrg._p(V), -1.0, 4, None, ctypes.byref(h)) == 1  # K <= 0
    bad = np.array([[1.0], [-0.5]])
    assert lib.ctmrg_init(2, 1, ctmrg._p(bad), 1.0, 4, None, ctypes.byref(h)) == 1  # not unit
    n = ctypes.c_size_t(0)
    assert lib.ctmrg_workspace_size(20, 512, None, ctypes.byref(n)) == 0
    assert n.value > 8 * (20 * 512) ** 2


def test_precision_option_is_validated_without_a_gpu_call():
    from paper_2004_08669_amd import ctmrg
    if not os.path.exists(ctmrg.LIB_PATH):
        pytest.skip("libctmrg.so not built")
    lib = ctmrg.load()
    o = ctmrg.default_options()
    assert o.precision == 0 and o.gap_tol == 1e-10
    n64, n32 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.ctmrg_workspace_size(20, 512, ctypes.byref(o), ctypes.byref(n64)) == 0
    o.precision = 1
    assert lib.ctmrg_workspace_size(20, 512, ctypes.byref(o), ctypes.byref(n32)) == 0
    # the mixed path adds FP32 copies of W, P, diag(omega) P and U
    N = 20 * 512
    assert n32.value - n64.value == 4 * (20 ** 4 + 3 * 512 * N)
    o.precision = 7
    assert lib.ctmrg_workspace_size(20, 512, ctypes.byref(o), ctypes.byref(n32)) == 1
    import numpy as np
    V = np.array([[1.0], [-1.0]])
    h = ctypes.c_void_p()
    assert lib.ctmrg_init(2, 1, ctmrg._p(V), 1.0, 4, ctypes.byref(o), ctypes.byref(h)) == 1


def test_derivative_entry_points_reject_bad_arguments_without_a_gpu_call():
    from paper_2004_08669_amd import ctmrg
    if not os.path.exists(ctmrg.LIB_PATH):
        pytest.skip("libctmrg.so not built")
    lib = ctmrg.load()
    d = ctmrg.Derivative()
    assert lib.ctmrg_fixed_point_derivative(None, 0, ctypes.byref(d)) == 1
    import numpy as np
    ob = np.zeros(3)
    kb = ctypes.c_double(0.0)
    assert lib.ctmrg_backward(None, ctmrg._p(ob), ctypes.byref(kb), None) == 1
