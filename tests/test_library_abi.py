"""The C-ABI library builds, loads without a GPU and exports every entry point that
include/ddrom.h declares; the Python binding refuses to run without the library."""
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2305_15163_amd", "libddrom.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ddrom.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?\**\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("dd_fom_residual", "ae_decode_hr", "ae_jacobian_hr", "sqp_step", "rom_solve_batch",
              "ddrom_model_create", "ddrom_workspace_create", "ddrom_last_error", "rom_solve_multi", "ddrom_autotune",
              "rom_solve_warm", "mlp_proposal", "mlp_train_step", "ae_train_step", "rom_decode_states",
              "rom_relative_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2305_15163_amd.ddrom as d
    monkeypatch.setattr(d, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(d, "_lib", None)
    with pytest.raises(RuntimeError):
        d.lib()
