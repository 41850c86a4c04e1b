"""Invalid inputs refused on the host, before any device call, beyond those of the ABI tests: a box
whose edges are long enough but whose perpendicular width is too thin for rc + skin, a flipped
diagonal, parameter values just outside their ranges, NULL result pointers, and arrays shorter
than the library reads (checked by the bindings)."""
import ctypes

import numpy as np
import pytest

from synth import configs


@pytest.fixture(scope="module")
def rc():
    from paper_1902_09171_amd import rcell
    rcell.load()
    return rcell


def _expect(rc, code, params, cells, words):
    with pytest.raises(rc.RCellError) as e:
        rc.RCellBatch(params, cells)
    assert e.value.code == code, (code, str(e.value))
    msg = str(e.value)
    assert all(w in msg for w in words), msg


def test_box_shape_and_width(rc):
    p = configs.kg_params()
    c = configs.kg_cell([20] * 10, 2)
    flipped = np.array(c["H0"], float).copy()
    flipped[2, 2] = -flipped[2, 2]
    _expect(rc, rc.ERR_ARG, p, [c, dict(c, H0=flipped)], ["cell 1", "positive diagonal"])
    # the perpendicular width, not the edge length, decides: a strongly tilted box whose edges are
    # all long enough is still too thin for rc + skin
    w = 2.05 * (p["rc"] + p["skin"])
    tilted = np.array([[w, 0.0, 0.0], [0.0, w, 10.0 * w], [0.0, 0.0, w]])
    _expect(rc, rc.ERR_BOX, p, [dict(c, H0=tilted)], ["cell 0", "too small"])


def test_parameters_just_outside_their_ranges(rc):
    c = configs.kg_cell([20] * 10, 3)
    _expect(rc, rc.ERR_ARG, configs.kg_params(skin=-0.1), [c], [">= 0"])
    _expect(rc, rc.ERR_ARG, configs.cu_params(sc_m=0), [configs.cu_cell(5, ncell=4)], ["Sutton-Chen"])


def test_null_result_pointers(rc):
    from paper_1902_09171_amd import rsur
    ps = rc.params_struct(configs.kg_params())
    inits = (rc.CellInit * 1)()
    assert rc.load().rcell_create(ctypes.byref(ps), inits, 1, None, None) == rc.ERR_ARG
    assert rsur.load().rsur_create(8, 16, 1, 2, 2, 64, None, None) == rc.ERR_ARG


def test_binding_checks_array_lengths_before_the_library_reads_them(rc):
    # the library reads natoms rows of x and v: a shorter v at create, or x / v of another length
    # in set_state, are refused by the binding before any call
    c = configs.kg_cell([20] * 10, 6)
    with pytest.raises(ValueError, match="v has shape"):
        rc.RCellBatch(configs.kg_params(), [dict(c, v=np.asarray(c["v"])[:-1])])
    b = rc.RCellBatch.__new__(rc.RCellBatch)        # a batch of one 200-atom cell, never created
    b.ncells, b.natoms, b._h = 1, [200], None
    with pytest.raises(ValueError, match="200 atoms"):
        b.set_state(0, np.zeros((199, 3)), np.zeros((200, 3)), np.eye(3) * 9, np.eye(3), 0)
    with pytest.raises(IndexError):
        b.set_state(-1, np.zeros((200, 3)), np.zeros((200, 3)), np.eye(3) * 9, np.eye(3), 0)


def test_surrogate_binding_checks_parameter_and_normalisation_sizes(rc):
    from paper_1902_09171_amd import rsur
    net = rsur.Surrogate.__new__(rsur.Surrogate)     # never created: the checks come first
    net.din, net.dout, net.nparams, net._h = 8, 2, 100, None
    with pytest.raises(ValueError, match="99 parameters"):
        net.set_params(0, np.zeros(99))
    with pytest.raises(ValueError, match="normalisation sizes"):
        net.set_norm(np.zeros(8), np.ones(8), np.zeros(3), np.ones(2))
