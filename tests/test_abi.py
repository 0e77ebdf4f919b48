"""The C-ABI library loads and exports every symbol include/mfe.h declares.

CPU only: no call here reaches a GPU.  Argument checks that fail before any
HIP call are exercised; compute calls are left to the GPU tests.
"""
import ctypes
import os
import re

import pytest

from paper_1505_08023_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfe.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfe_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ("mfe_ctx_create", "mfe_problem_create", "mfe_spmv", "mfe_cg", "mfe_dot"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    # the binding declares exactly the header's functions
    assert set(_lib.SIGNATURES) == set(declared_functions())


def test_version_and_error_string():
    lib = _lib.load()
    assert lib.mfe_version() == 13
    assert isinstance(lib.mfe_last_error(), bytes)


def test_argument_checks_before_any_device_call():
    lib = _lib.load()
    out = ctypes.c_void_p()
    assert lib.mfe_ctx_create(0, None, _lib.mfe_alloc_fn(), _lib.mfe_free_fn(), None, None) == _lib.MFE_EINVAL
    assert b"out" in lib.mfe_last_error()
    # one callback without the other
    cb = _lib.mfe_alloc_fn(lambda n, u: None)
    assert lib.mfe_ctx_create(0, None, cb, _lib.mfe_free_fn(), None, ctypes.byref(out)) == _lib.MFE_EINVAL
    assert lib.mfe_problem_create(None, 4, 4, 4, None, None, 1, 1, ctypes.byref(out)) == _lib.MFE_EINVAL
    assert lib.mfe_problem_from_csr(None, 4, None, None, None, None, 1, 1, ctypes.byref(out)) == _lib.MFE_EINVAL
    assert lib.mfe_spmv(None, 1, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_spmv_f32(None, 1, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_cg(None, 1, None, 1e-8, 10, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_dot(None, 1, None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_spmv_dot_noalloc(None, 1, None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_stream_probe(None, 0, 1, None, None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_problem_set_bc(None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_problem_info(None, None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_problem_bcrs13_layout(None, None, None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_problem_csr_layout(None, None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_problem_csr_groups(None, None, None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_batch_bcrs13_layout(None, None, None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_problem_export_csr(None, None, None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_net_loss_grad_energy(None, None, 1, 1, None, None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_cg_mixed_ex(None, 1, None, 1e-8, 1e-4, 10, 10, 0, None) == _lib.MFE_EINVAL
    assert lib.mfe_batch_cg_mixed_ex(None, 1, None, 1e-8, 1e-4, 10, 10, 0, None) == _lib.MFE_EINVAL
    assert lib.mfe_net_set_grad(None, None) == _lib.MFE_EINVAL
    assert lib.mfe_rhs(None, None) == _lib.MFE_EINVAL
    assert lib.mfe_prolong_trilinear(None, 4, 4, 4, None, 2, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_problem_from_csr_host(None, 4, None, None, None, None, 1, 1, ctypes.byref(out)) == _lib.MFE_EINVAL
    assert lib.mfe_problem_export_csr_host(None, None, None, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_batch_from_problems(None, 1, None, 1, 1, ctypes.byref(out)) == _lib.MFE_EINVAL
    assert lib.mfe_cg_batched(None, 1, None, 1, None, 1e-8, 10, 0, None) == _lib.MFE_EINVAL
    assert lib.mfe_conv3d_dgrad_bf16(None, 0, 1, 9, 8, None, 16, None, 0, None, None) == _lib.MFE_EINVAL
    assert lib.mfe_problem_destroy(None) == _lib.MFE_OK
    assert lib.mfe_ctx_destroy(None) == _lib.MFE_OK


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libmfe.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load()
