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


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a header struct, from a C program compiled against include/ctmrg.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    body = "".join(f'    printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src.write_text(f'#include <stdio.h>\n#include <stddef.h>\n#include "ctmrg.h"\nint main(void) {{\n'
                   f'    printf("%zu\\n", sizeof({struct}));\n{body}    return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    return out[0], out[1:]


@pytest.mark.parametrize("struct,cls", [("ctmrg_options", "Options"), ("ctmrg_observables_t", "Observables"),
                                        ("ctmrg_derivative_t", "Derivative")])
def test_binding_structs_match_the_header(struct, cls, tmp_path):
    """The ctypes structures of the binding have the header's fields, in order, at the same offsets,
    and the same size (what a C caller and the Python binding exchange)."""
    from paper_2004_08669_amd import ctmrg
    C = getattr(ctmrg, cls)
    names = [n for n, _ in C._fields_]
    size, offsets = _c_layout(struct, names, tmp_path)
    assert size == ctypes.sizeof(C)
    assert offsets == [getattr(C, n).offset for n in names]
    # and the header has no field the binding lacks
    text = open(os.path.join(ROOT, "include", "ctmrg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    m = re.search(r"typedef struct[^{]*\{([^}]*)\}\s*" + re.escape(struct) + r"\s*;", text)
    assert m, struct
    declared = re.findall(r"([A-Za-z_][A-Za-z0-9_]*)\s*;", m.group(1))
    assert declared == names
