"""The C-ABI library loads on the host and exports every entry point of include/flare.h
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flare.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\s*\*)\s*(flare_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_four_path_calls():
    names = declared()
    for n in ["flare_neighbors", "flare_descriptors", "flare_energy_forces", "flare_variance"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2204_12573_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = binding.load()
    for name in declared():
        assert hasattr(lib, name), name
    assert set(declared()) == set(binding.SIGNATURES)


def declared_arities():
    """Number of parameters of every declared entry point (no function-pointer arguments)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"^\s*(?:int|const char\s*\*)\s*(flare_\w+)\s*\(([^)]*)\)\s*;", text, flags=re.M):
        params = m.group(2).strip()
        out[m.group(1)] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_argument_counts_match_the_header():
    from paper_2204_12573_amd import binding
    ar = declared_arities()
    assert set(ar) == set(declared())
    for name, (_, args) in binding.SIGNATURES.items():
        assert len(args) == ar[name], (name, len(args), ar[name])


def test_host_only_calls():
    from paper_2204_12573_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = binding.load()
    assert lib.flare_strerror(-4).decode() == "capacity exceeded"
    # argument checks run before any device work
    assert lib.flare_model_create(None, 2, 8, 3, 4.5, None, None, 0) == binding.E_ARG
    assert b"null" in lib.flare_last_error()
    h = ctypes.c_void_p()
    dummy = (ctypes.c_double * 4)()
    assert lib.flare_model_create(ctypes.byref(h), 3, 8, 3, 4.5, dummy, dummy, 0) == binding.E_UNSUPPORTED
    assert lib.flare_neighbors(None, 1, None, None, None, None, 1, None, None, 0.2) == binding.E_ARG
    assert lib.flare_virial(None, None) == binding.E_ARG
    assert lib.flare_model_create(ctypes.byref(h), 2, 8, 3, 4.5, dummy, dummy, 4) == binding.E_UNSUPPORTED
