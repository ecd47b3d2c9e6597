"""CPU-side checks of the C-ABI library: it is built for gfx950, loads, and
exports every entry point that include/hafgpu.h declares.  No compute calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hafgpu.h")
LIB = os.path.join(ROOT, "paper_1805_12498_amd", "libhafgpu.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(haf\w*|lhaf\w*|perm\w*)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1805_12498_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("haf_c128", "lhaf_c128", "haf_c128_dev", "lhaf_c128_dev", "haf_batched_c128", "haf_server_create",
                 "haf_server_submit", "haf_server_poll", "haf_terms_dev", "haf_last_error"):
        assert must in names, must


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_1805_12498_amd import _native
    assert sorted(_native.EXPORTS) == declared_functions()


def test_library_targets_gfx950():
    """The fat binary carries a gfx950 code object (offload target id in the bundle)."""
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_version_without_gpu(lib):
    lib.haf_version.restype = ctypes.c_char_p
    assert lib.haf_version().startswith(b"hafgpu")


@pytest.mark.parametrize("value,expect", [("65536", 65536), ("64M", 64 << 20), ("2G", 2 << 30), ("junk", 1 << 30)])
def test_server_arena_from_environment(lib, monkeypatch, value, expect):
    """HAF_ARENA_BYTES sets the default server arena (host-only call, no device)."""
    from paper_1805_12498_amd._native import ServerConfig
    monkeypatch.setenv("HAF_ARENA_BYTES", value)
    cfg = ServerConfig()
    lib.haf_server_default_config(ctypes.byref(cfg))
    assert cfg.arena_bytes == expect


def test_batched_cache_needs_its_variable(lib, monkeypatch):
    """Without HAF_AUTOTUNE_CACHE the cache loader reports HAF_E_STATE (host-only)."""
    monkeypatch.delenv("HAF_AUTOTUNE_CACHE", raising=False)
    lib.haf_last_error.restype = ctypes.c_char_p
    assert lib.haf_batched_load_cache() == 8
    assert b"HAF_AUTOTUNE_CACHE" in lib.haf_last_error()
