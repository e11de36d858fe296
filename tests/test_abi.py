"""The C ABI library loads and exports every function include/flashsplat.h
declares; host-side argument checks work without a GPU (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flashsplat.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fs_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (binds the library to torch's HIP runtime)
    from paper_2409_08270_amd import _lib as L
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 13
    from paper_2409_08270_amd import _lib as L
    assert sorted(L.EXPORTS) == sorted(set(L.EXPORTS))
    for n in names:
        assert hasattr(lib, n), f"{n} declared in the header but not exported"
        assert n in L.EXPORTS, f"{n} not bound in the Python binding"


def test_defaults_and_host_side_validation(lib):
    from paper_2409_08270_amd import _lib as L
    p = L.params()
    assert (p.tile_w, p.tile_h) == (16, 16)
    assert p.sigma_k == 3.0 and abs(p.lowpass - 0.3) < 1e-7 and abs(p.alpha_min - 1 / 255) < 1e-9
    e = L.params_exact()
    assert e.alpha_min == 0.0 and e.alpha_max == 1.0 and e.t_min == 0.0
    # NULL context is rejected before anything touches a device
    assert lib.fs_assign(None, None, None, 0, 2, 0.0, None, None) == L.FS_ERR_ARG
    assert lib.fs_project(None, None, None, 0, None, None) == L.FS_ERR_ARG
    assert lib.fs_ctx_destroy(None) == L.FS_ERR_ARG
    assert lib.fs_error_string(L.FS_ERR_CAPACITY) == b"output capacity too small"
    st = L.FsStatus()
    assert lib.fs_status_get(None, ctypes.byref(st), 0) == L.FS_ERR_ARG
