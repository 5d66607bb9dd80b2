"""CPU-side checks of the C ABI: the library loads and exports every entry point that
include/pcprop.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcprop.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\*|size_t)\s+(pc_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("pc_propagate", "pc_propagate_batched", "pc_ctx_create", "pc_workspace_bytes",
                 "pc_get_operator", "pc_eval_force"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2301_03989_amd import build
    build.ensure_built()
    lib = ctypes.CDLL(build.LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_the_same_symbols():
    pytest.importorskip("torch")
    from paper_2301_03989_amd import pcprop
    assert sorted(pcprop.EXPORTS) == declared_functions()


def test_version_and_strerror_without_gpu():
    from paper_2301_03989_amd import build
    build.ensure_built()
    lib = ctypes.CDLL(build.LIB)
    assert lib.pc_version() == 100
    lib.pc_strerror.restype = ctypes.c_char_p
    assert lib.pc_strerror(0) == b"ok"
    assert b"workspace" in lib.pc_strerror(5)


def test_context_creation_fails_cleanly_without_gpu():
    # pc_ctx_create needs a device; without one it must fail cleanly, not crash
    from paper_2301_03989_amd import build
    build.ensure_built()
    lib = ctypes.CDLL(build.LIB)
    h = ctypes.c_void_p()
    rc = lib.pc_ctx_create(0, ctypes.byref(h))
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if not has_gpu:
        assert rc == 1 and not h.value
    elif rc == 0:
        lib.pc_ctx_destroy(h)


def test_default_opts_fill_the_binding_struct_exactly():
    """pc_default_opts writes every field of the binding's pc_opts and nothing past it:
    the ctypes layout and the header's agree (a field missing on either side shifts or
    overruns the sentinel bytes)."""
    pytest.importorskip("torch")
    from paper_2301_03989_amd import build, pcprop
    build.ensure_built()
    lib = ctypes.CDLL(build.LIB)
    n = ctypes.sizeof(pcprop._Opts)
    buf = (ctypes.c_ubyte * (n + 64))(*([0xAB] * (n + 64)))
    lib.pc_default_opts(ctypes.byref(buf))
    assert bytes(buf[n:]) == b"\xab" * 64
    o = pcprop._Opts.from_buffer_copy(bytes(buf[:n]))
    d = pcprop.Context.opts()
    for name, _ in pcprop._Opts._fields_:
        assert getattr(o, name) == getattr(d, name), name
    assert o.conv == pcprop.CONV["ic"] and o.max_iter == 64
