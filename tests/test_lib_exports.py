"""The C ABI library loads and exports every function declared in include/msc.h (no GPU
work is done)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(msc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("msc_op_create_csr", "msc_op_set_shifts", "msc_solve", "msc_solve_adjoint",
                     "msc_solve_batched", "msc_op_destroy", "msc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1102_2143_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmsc.so is not built: run `python -m paper_1102_2143_amd.build`")
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(_lib.EXPORTED) == set(declared_functions())
    assert lib.msc_version().decode().startswith("msc")


def test_params_default_and_struct_layout():
    import ctypes
    from paper_1102_2143_amd import _lib
    lib = _lib.load()
    p = _lib.Params()
    lib.msc_params_default(ctypes.byref(p))
    assert p.tol == 1e-10 and p.max_iter == 10000 and p.reliable_every == 50
    assert p.poll_every == 16 and p.verify == 1
    assert p.update_steps == 8 and p.sweep == 0
    assert ctypes.sizeof(_lib.Params) == 80  # update_steps and the sweep order appended
    assert ctypes.sizeof(_lib.Info) == 160  # FP64-phase timing fields appended


def test_null_arguments_are_rejected_without_gpu_work():
    import ctypes
    from paper_1102_2143_amd import _lib
    lib = _lib.load()
    assert lib.msc_op_create_csr(None, 0, 10, 10, None, None, None, None) == _lib.MSC_EINVAL
    assert "NULL" in _lib.last_error()
    h = ctypes.c_void_p()
    assert lib.msc_op_create_csr(ctypes.byref(h), 7, 10, 10, None, None, None, None) == _lib.MSC_EINVAL
    assert lib.msc_op_create_csr(ctypes.byref(h), 0, 0, 0, None, None, None, None) == _lib.MSC_EINVAL
    assert lib.msc_op_set_shifts(None, None, 1) == _lib.MSC_EINVAL
    assert lib.msc_solve(None, None, None, None, None, None) == _lib.MSC_EINVAL
    lib.msc_op_destroy(None)
