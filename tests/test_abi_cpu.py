"""CPU-side checks of the C-ABI library: it loads without a GPU and exports
every entry point that include/ckks.h declares (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ckks.h")
LIB = os.path.join(ROOT, "paper_2606_10477_amd", "libckks_hip.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(ckks_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for n in ["ckks_ctx_create", "ckks_keygen", "ckks_encrypt", "ckks_decrypt", "ckks_hmult_relin",
              "ckks_rescale", "ckks_rotate", "ckks_cheb_eval", "ckks_bootstrap", "ckks_invsqrt"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_every_declared_symbol():
    from paper_2606_10477_amd import ckks
    assert set(declared_functions()) <= set(ckks.SIGNATURES)
