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


def test_create_rejects_bad_parameters_and_cells_on_the_host(lib):
    # each rejection happens before any device call (no context is left behind, none is needed)
    import numpy as np
    from paper_1902_09171_amd import rcell
    from synth import configs
    L = rcell.load()
    cell = configs.kg_cell([20] * 10, 7)
    x = np.ascontiguousarray(cell["x"], np.float64)
    H0 = np.ascontiguousarray(cell["H0"], np.float64)

    def create(p, natoms=len(x), H=H0):
        init = (rcell.CellInit * 1)()
        init[0].natoms = natoms
        init[0].nbonds = 0
        init[0].H0 = H.ctypes.data
        init[0].x = x.ctypes.data
        out = ctypes.c_void_p()
        code = L.rcell_create(ctypes.byref(rcell.params_struct(p)), init, 1, None, ctypes.byref(out))
        assert out.value is None
        return code, L.rcell_last_error(None).decode()

    kg = configs.kg_params()
    cases = [
        (dict(kg, potential=7), rcell.ERR_ARG, "unknown potential"),
        (dict(kg, precision=5), rcell.ERR_ARG, "unknown precision"),
        (dict(kg, dt=0.0), rcell.ERR_ARG, "dt"),
        (dict(kg, lj_sigma=0.0), rcell.ERR_ARG, "lj_sigma"),
        (configs.cu_params(sc_n=40), rcell.ERR_ARG, "Sutton-Chen"),
    ]
    for p, code, words in cases:
        got, msg = create(p)
        assert got == code and words in msg, (p, got, msg)
    got, msg = create(kg, natoms=0)
    assert got == rcell.ERR_ARG and "cell 0" in msg
    sheared = H0.copy()
    sheared[1, 0] = 0.5                                  # below the diagonal: not upper triangular
    got, msg = create(kg, H=np.ascontiguousarray(sheared))
    assert got == rcell.ERR_ARG and "upper triangular" in msg
    got, msg = create(dict(kg, skin=0.5 * H0[0, 0]))     # rc + skin beyond half the box width
    assert got == rcell.ERR_BOX and "box too small" in msg


def test_surrogate_create_rejects_bad_shapes_on_the_host(lib):
    from paper_1902_09171_amd import rcell
    L = rcell.load()
    L.rsur_last_error.restype = ctypes.c_char_p
    for din, width, depth, dout, K, B in ((0, 256, 4, 6, 5, 256), (153, 256, 4, 0, 5, 256), (153, 0, 4, 6, 5, 256),
                                          (153, 256, -1, 6, 5, 256), (153, 256, 4, 6, 0, 256), (153, 256, 4, 6, 5, 0)):
        out = ctypes.c_void_p()
        code = L.rsur_create(din, width, depth, dout, K, B, None, ctypes.byref(out))
        assert code == rcell.ERR_ARG and out.value is None, (din, width, depth, dout, K, B)
        assert b"din, dout, ensemble" in L.rsur_last_error(None)
