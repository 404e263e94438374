"""The C-ABI library loads and exports every entry point include/ipc.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ipc.h")
LIB = os.path.join(ROOT, "paper_2503_05020_amd", "libipc_mi355x.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ipc_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["ipc_create_scene", "ipc_step", "ipc_step_batch", "ipc_get_state", "ipc_set_state",
              "ipc_destroy_scene", "ipc_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_every_export():
    from paper_2503_05020_amd import ipc
    assert sorted(ipc.EXPORTS) == declared()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2503_05020_amd import ipc
    monkeypatch.setattr(ipc, "_lib", None)
    monkeypatch.setattr(ipc, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        ipc.lib()


def test_binding_constants_match_header():
    """Every integer #define of include/ipc.h that the binding also names has the same value."""
    from paper_2503_05020_amd import ipc
    src = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(IPC_\w+)\s+\(?(-?\d+)\)?\s*$", src, flags=re.M))
    shared = [n for n in defs if hasattr(ipc, n)]
    assert "IPC_TUNE_COARSE" in shared and "IPC_COARSE_BODIES" in shared
    for n in shared:
        assert getattr(ipc, n) == int(defs[n]), n
