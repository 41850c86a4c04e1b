"""The C-ABI library loads on the CPU and exports every function its headers declare.
No compute call is made (there may be no GPU)."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1902_09171_amd", "librcell.so")


def declared():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(r(?:cell|sur)_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1902_09171_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "rcell_create" in names and "rcell_run" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, flags=re.M), n


def test_binding_lists_match_header():
    from paper_1902_09171_amd import rcell, rsur
    decl = [n for n in declared() if n.startswith("rcell_")]
    assert sorted(rcell.EXPORTS) == decl
    assert sorted(rsur.EXPORTS) == [n for n in declared() if n.startswith("rsur_")]


def test_create_rejects_bad_arguments_without_touching_the_gpu(lib):
    # argument validation happens on the host before any device call
    from paper_1902_09171_amd import rcell
    from synth import configs
    p = rcell.params_struct(configs.kg_params())
    out = ctypes.c_void_p()
    L = rcell.load()
    assert L.rcell_create(ctypes.byref(p), None, 0, None, ctypes.byref(out)) == rcell.ERR_ARG
    assert out.value is None
    assert b"ncells" in L.rcell_last_error(None)
