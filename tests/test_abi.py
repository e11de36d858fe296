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


def test_batch_defaults_and_null_handling(lib):
    from paper_2409_08270_amd import _lib as L
    o = L.batch_opts()
    assert (o.pair_budget, o.elem_budget, o.zero_accumulators, o.use_graph, o.reduction) == (0, 0, 1, 1, L.FS_RED_AUTO)
    assert (o.depth_slabs, o.lanes) == (0, 0)
    out = ctypes.c_void_p()
    assert lib.fs_batch_create(None, None, 0, None, None, ctypes.byref(out)) == L.FS_ERR_ARG
    assert lib.fs_batch_run(None) == L.FS_ERR_ARG
    assert lib.fs_batch_destroy(None) == L.FS_ERR_ARG
    inf = L.FsBatchInfo()
    assert lib.fs_batch_get_info(None, ctypes.byref(inf)) == L.FS_ERR_ARG
    ms, cnt = ctypes.c_float(), ctypes.c_int32()
    assert lib.fs_batch_accumulate_ms(None, ctypes.byref(ms), ctypes.byref(cnt)) == L.FS_ERR_ARG
    ci = L.FsChunkInfo()
    assert lib.fs_batch_chunk_lists(None, 0, None, 0, None, 0, None, 0, ctypes.byref(ci)) == L.FS_ERR_ARG


def test_header_limits_match_the_binding():
    from paper_2409_08270_amd import _lib as L
    src = open(HEADER).read()
    for name in ("FS_NOALLOC_MAX_VIEWS", "FS_NOALLOC_MAX_TILES", "FS_DEV_MANY_LABELS", "FS_RED_PLAIN", "FS_RED_LDS",
                 "FS_RED_LDS2SUM", "FS_RED_DET"):
        m = re.search(r"#define\s+" + name + r"\s+(\d+)", src)
        assert m and int(m.group(1)) == getattr(L, name), name


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof/offsetof of every public struct, from a C compiler, against the ctypes mirror."""
    import subprocess
    from paper_2409_08270_amd import _lib as L
    structs = {"fs_gaussians": L.FsGaussians, "fs_camera": L.FsCamera, "fs_params": L.FsParams,
               "fs_proj": L.FsProj, "fs_bins": L.FsBins, "fs_pixel_out": L.FsPixelOut, "fs_status": L.FsStatus,
               "fs_scene": L.FsScene, "fs_batch_opts": L.FsBatchOpts, "fs_batch_info": L.FsBatchInfo,
               "fs_chunk_info": L.FsChunkInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.split("\n") if l)
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, f"{cname}.{f}"
