"""The C-ABI library loads without a GPU and exports every entry point that
include/mcdi.h declares (no compute calls)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcdi.h")
LIB = os.path.join(ROOT, "paper_2206_03380_amd", "libmcdi.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(mcdi_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    names = declared()
    assert "mcdi_shade_fwd" in names and "mcdi_build_env_cdf" in names and len(names) >= 12
    lib = ctypes.CDLL(LIB)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_version_and_binding_list():
    lib = ctypes.CDLL(LIB)
    lib.mcdi_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.mcdi_version()
    from paper_2206_03380_amd import _lib
    assert set(_lib.EXPORTED) <= set(declared())


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_validation_without_device():
    """Argument validation runs before any device work: calls with bad
    arguments return MCDI_E_INVALID / MCDI_E_UNSUPPORTED on a machine without
    a GPU, and mcdi_last_error names the call."""
    from paper_2206_03380_amd import _lib as L
    lib = L.lib()
    out = ctypes.c_void_p()
    assert lib.mcdi_build_scene(None, 3, None, 1, None, None, ctypes.byref(out)) == L.MCDI_E_INVALID
    assert b"mcdi_build_scene" in lib.mcdi_last_error()
    assert lib.mcdi_build_scene(None, -1, None, 0, None, None, ctypes.byref(out)) == L.MCDI_E_INVALID
    assert lib.mcdi_build_scene(None, 0, None, 1 << 27, None, None, ctypes.byref(out)) == L.MCDI_E_UNSUPPORTED
    assert lib.mcdi_build_scene(None, 0, None, 1 << 26, None, None, ctypes.byref(out)) == L.MCDI_E_UNSUPPORTED
    assert lib.mcdi_build_env_cdf(None, 4, 4, None, None, ctypes.byref(out)) == L.MCDI_E_INVALID
    assert lib.mcdi_build_env_cdf(ctypes.c_void_p(16), 5000, 4, None, None, ctypes.byref(out)) == L.MCDI_E_UNSUPPORTED
    assert lib.mcdi_build_env_cdf(ctypes.c_void_p(16), 0, 4, None, None, ctypes.byref(out)) == L.MCDI_E_INVALID
    g = L.GBuffer()
    p = L.Params(4, 0, 0, 1.0, 1e-3, None)
    assert lib.mcdi_shade_fwd(None, None, ctypes.byref(g), ctypes.byref(p), None, None, None, None, None) == L.MCDI_E_INVALID
    n = ctypes.c_int32()
    assert lib.mcdi_trace_times(None, 4, ctypes.byref(n)) == L.MCDI_E_INVALID
    assert lib.mcdi_trace_anyhit(None, None, None, 0, None, 0, None) == L.MCDI_E_INVALID
    # edge list and edge-sampled visibility gradient
    assert lib.mcdi_build_edges(None, 3, 10, None, None, None) == L.MCDI_E_INVALID
    assert lib.mcdi_build_edges(None, 3, 10, None, None, ctypes.byref(out)) == L.MCDI_E_INVALID
    assert b"mcdi_build_edges" in lib.mcdi_last_error()
    assert lib.mcdi_build_edges(None, -1, 10, None, None, ctypes.byref(out)) == L.MCDI_E_INVALID
    assert lib.mcdi_build_edges(None, 1 << 26, 10, None, None, ctypes.byref(out)) == L.MCDI_E_UNSUPPORTED
    assert lib.mcdi_build_edges(None, 0, 1 << 31, None, None, ctypes.byref(out)) == L.MCDI_E_UNSUPPORTED
    cnt = ctypes.c_int64()
    assert lib.mcdi_edges_count(None, ctypes.byref(cnt)) == L.MCDI_E_INVALID
    assert lib.mcdi_edges_copy(None, None, None) == L.MCDI_E_INVALID
    assert lib.mcdi_shade_bwd_edges(None, None, None, None, 0, ctypes.byref(g), ctypes.byref(p), 4, 1, None, None,
                                    None, None, None) == L.MCDI_E_INVALID
    assert b"mcdi_shade_bwd_edges" in lib.mcdi_last_error()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library the loader raises, and host tensors are
    refused before any call: there is no fallback path."""
    import torch
    import paper_2206_03380_amd as M
    from paper_2206_03380_amd import _lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "libmcdi.so"))
    with pytest.raises(ImportError, match="no fallback"):
        L.lib()
    verts = torch.zeros((3, 3))
    tris = torch.zeros((1, 3), dtype=torch.int32)
    with pytest.raises(TypeError, match="CUDA"):
        M.Scene(verts, tris)


def test_binding_structs_match_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (the header compiled by the host C compiler)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    from paper_2206_03380_amd import _lib as L
    pairs = {"Allocator": "mcdi_allocator", "GBuffer": "mcdi_gbuffer", "Params": "mcdi_params",
             "Stats": "mcdi_stats", "SceneInfo": "mcdi_scene_info_t", "BilateralGuide": "mcdi_bilateral_guide",
             "ServerConfig": "mcdi_server_config", "Request": "mcdi_request", "ServerInfo": "mcdi_server_info_t"}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mcdi.h"', "int main(void) {"]
    want = []
    for py, c in pairs.items():
        cls = getattr(L, py)
        lines.append('printf("%%zu\\n", sizeof(%s));' % c)
        want.append(ctypes.sizeof(cls))
        for name, _ in cls._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (c, name))
            want.append(getattr(cls, name).offset)
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == want
