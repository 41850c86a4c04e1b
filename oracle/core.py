"""ctypes wrapper around the FP64 C oracle (rcell_oracle.c).  Test infrastructure only.

`build()` compiles liboracle.so with gcc (-O2, OpenMP over cells, no intrinsics).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rcell_oracle.c")
_HDR = os.path.join(_HERE, "rcell_oracle.h")
_LIB = os.environ.get("RCELL_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

POTENTIALS = {"kg": 1, "sc_eam": 2}
OK, ERR_ARG, ERR_BAD_F, ERR_BOX, ERR_BOND, ERR_NONFINITE, ERR_OOM, ERR_STATE = 0, -1, -2, -3, -4, -5, -6, -8


class OracleError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"oracle error {code} {msg}")
        self.code = code


def build(force: bool = False) -> str:
    if os.environ.get("RCELL_ORACLE_LIB"):
        return _LIB                      # a prebuilt variant (mutation tests)
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_HDR))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("potential", ctypes.c_int32), ("include_kinetic", ctypes.c_int32),
                ("dt", ctypes.c_double), ("temperature", ctypes.c_double), ("gamma", ctypes.c_double),
                ("mass", ctypes.c_double), ("kB", ctypes.c_double), ("mvv2e", ctypes.c_double),
                ("rc", ctypes.c_double), ("skin", ctypes.c_double),
                ("lj_eps", ctypes.c_double), ("lj_sigma", ctypes.c_double),
                ("fene_K", ctypes.c_double), ("fene_R0", ctypes.c_double),
                ("sc_eps", ctypes.c_double), ("sc_a", ctypes.c_double), ("sc_c", ctypes.c_double),
                ("sc_n", ctypes.c_int32), ("sc_m", ctypes.c_int32), ("seed", ctypes.c_uint64)]


def params_struct(p: dict) -> _Params:
    s = _Params()
    for name, _ in _Params._fields_:
        val = p[name]
        if name == "potential":
            val = POTENTIALS[val] if isinstance(val, str) else int(val)
        setattr(s, name, val)
    return s


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "orc_qr": [vp, vp, vp], "orc_lattice_reduce": [vp], "orc_philox4x32_10": [vp, vp, vp],
            "orc_pairs": [vp, i32, vp, d, i64, vp, vp, vp],
            "orc_stress_to_fem": [vp, vp, vp, vp],
            "orc_forces": [vp, vp, i32, vp, i32, vp, vp, vp, vp],
            "orc_create": [vp, i32, vp, vp, vp, vp, vp, vp, vp],
            "orc_set_deformation": [vp, vp], "orc_run": [vp, i32], "orc_get_stress": [vp, vp, vp],
            "orc_set_cell_ids": [vp, vp],
            "orc_minimize": [vp, i32, ctypes.c_double, vp],
            "orc_get_status": [vp, vp], "orc_get_forces": [vp, i32, vp],
            "orc_get_state": [vp, i32, vp, vp, vp, vp, vp],
            "orc_set_state": [vp, i32, vp, vp, vp, vp, i64], "orc_get_energy": [vp, vp, vp],
            "orc_get_box": [vp, i32, vp, vp, vp, vp], "orc_last_error": [vp], "orc_destroy": [vp],
            "orc_threads": [i32],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.orc_lattice_reduce.restype = None
        L.orc_philox4x32_10.restype = None
        L.orc_destroy.restype = None
        L.orc_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a.reshape(shape) if shape is not None else a


def threads(n: int = 0) -> int:
    return lib().orc_threads(n)


def qr(F):
    F = _f64(F, (3, 3))
    Q, R = np.zeros((3, 3)), np.zeros((3, 3))
    st = lib().orc_qr(_p(F), _p(Q), _p(R))
    if st != OK:
        raise OracleError(st, "qr")
    return Q, R


def lattice_reduce(H):
    H = _f64(H, (3, 3)).copy()
    lib().orc_lattice_reduce(_p(H))
    return H


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def pairs(H, x, rc):
    H = _f64(H, (3, 3))
    x = _f64(x, (-1, 3))
    n = len(x)
    npairs = ctypes.c_int64(0)
    dummy_i, dummy_d = np.zeros(2, np.int32), np.zeros(3)
    st = lib().orc_pairs(_p(H), n, _p(x), rc, 0, _p(dummy_i), _p(dummy_d), ctypes.byref(npairs))
    if st != OK:
        raise OracleError(st, "pairs")
    m = npairs.value
    ij, d = np.zeros((max(m, 1), 2), np.int32), np.zeros((max(m, 1), 3))
    st = lib().orc_pairs(_p(H), n, _p(x), rc, m, _p(ij), _p(d), ctypes.byref(npairs))
    return ij[:m], d[:m]


def forces(params, H, x, bonds=None):
    """Conservative forces, potential energy and pair virial W (3x3) in any box H."""
    ps = params_struct(params)
    H = _f64(H, (3, 3))
    x = _f64(x, (-1, 3))
    b = np.ascontiguousarray(np.zeros((0, 2), np.int32) if bonds is None else np.asarray(bonds, np.int32))
    f = np.zeros_like(x)
    pe = ctypes.c_double(0.0)
    W = np.zeros((3, 3))
    st = lib().orc_forces(ctypes.byref(ps), _p(H), len(x), _p(x), len(b), _p(b) if len(b) else None,
                          _p(f), ctypes.byref(pe), _p(W))
    if st != OK:
        raise OracleError(st, "forces")
    return f, pe.value, W


def stress_to_fem(F, sigma_md6):
    F = _f64(F, (3, 3))
    s = _f64(sigma_md6, (6,))
    out, P = np.zeros(6), np.zeros((3, 3))
    st = lib().orc_stress_to_fem(_p(F), _p(s), _p(out), _p(P))
    if st != OK:
        raise OracleError(st, "stress_to_fem")
    return out, P


class OracleBatch:
    """Batched r-cell context with the library's create / set_deformation / run / get_stress
    semantics, computed by the FP64 oracle."""

    def __init__(self, params, cells, cell_ids=None):
        """cell_ids: the cells' indices in the Langevin noise counter (default 0..n-1), e.g. their
        positions in a larger batch of which these cells are a sample."""
        self.params = dict(params)
        self._ps = params_struct(params)
        self.natoms = np.array([len(c["x"]) for c in cells], np.int32)
        bl = [np.asarray(c.get("bonds", np.zeros((0, 2))), np.int32).reshape(-1, 2) for c in cells]
        self.nbonds = np.array([len(b) for b in bl], np.int32)
        self.ncells = len(cells)
        H0 = _f64(np.stack([c["H0"] for c in cells]) if cells else np.zeros((0, 3, 3)))
        x = _f64(np.concatenate([c["x"] for c in cells]) if cells else np.zeros((0, 3)))
        # cells without velocities: all of them draw Maxwell-Boltzmann velocities from the seed
        no_v = [c.get("v") is None for c in cells]
        if any(no_v) and not all(no_v):
            raise ValueError("either every cell or no cell comes without velocities")
        v = None if (cells and all(no_v)) else _f64(
            np.concatenate([c["v"] for c in cells]) if cells else np.zeros((0, 3)))
        b = np.ascontiguousarray(np.concatenate(bl) if bl else np.zeros((0, 2), np.int32))
        h = ctypes.c_void_p()
        st = lib().orc_create(ctypes.byref(self._ps), self.ncells, _p(self.natoms), _p(self.nbonds),
                              _p(H0), _p(x), _p(v), _p(b) if len(b) else None, ctypes.byref(h))
        if st != OK:
            raise OracleError(st, "create")
        self._h = h
        if cell_ids is not None:
            ids = np.ascontiguousarray(cell_ids, np.int32)
            assert len(ids) == self.ncells
            st = lib().orc_set_cell_ids(self._h, _p(ids))
            if st != OK:
                raise OracleError(st, "set_cell_ids")

    def __del__(self):
        # at interpreter exit the module's globals may already be gone: then the process is ending
        # and its memory is released with it
        if getattr(self, "_h", None) and _lib is not None and callable(lib):
            _lib.orc_destroy(self._h)
            self._h = None

    def _check(self, st, what):
        if st != OK:
            raise OracleError(st, what + ": " + (lib().orc_last_error(self._h) or b"").decode())

    def set_deformation(self, F):
        F = _f64(F, (self.ncells, 3, 3))
        self._check(lib().orc_set_deformation(self._h, _p(F)), "set_deformation")

    def run(self, nsteps):
        self._check(lib().orc_run(self._h, int(nsteps)), "run")

    def minimize(self, max_iter, ftol):
        """Molecular statics by FIRE (see orc_minimize); returns the iterations used per cell."""
        iters = np.zeros(self.ncells, np.int32)
        self._check(lib().orc_minimize(self._h, int(max_iter), float(ftol), _p(iters)), "minimize")
        return iters

    def get_stress(self, with_P=False):
        s = np.zeros((self.ncells, 6))
        P = np.zeros((self.ncells, 3, 3)) if with_P else None
        self._check(lib().orc_get_stress(self._h, _p(s), _p(P)), "get_stress")
        return (s, P) if with_P else s

    def status(self):
        s = np.zeros(self.ncells, np.int32)
        lib().orc_get_status(self._h, _p(s))
        return s

    def get_forces(self, cell):
        f = np.zeros((self.natoms[cell], 3))
        self._check(lib().orc_get_forces(self._h, cell, _p(f)), "get_forces")
        return f

    def get_state(self, cell):
        n = self.natoms[cell]
        x, v, H, Rp = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((3, 3)), np.zeros((3, 3))
        step = ctypes.c_int64(0)
        self._check(lib().orc_get_state(self._h, cell, _p(x), _p(v), _p(H), _p(Rp), ctypes.byref(step)),
                    "get_state")
        return dict(x=x, v=v, H=H, Rprev=Rp, step=step.value)

    def set_state(self, cell, x, v, H, Rprev, step):
        x, v, H, Rp = _f64(x), _f64(v), _f64(H, (3, 3)), _f64(Rprev, (3, 3))
        self._check(lib().orc_set_state(self._h, cell, _p(x), _p(v), _p(H), _p(Rp), int(step)), "set_state")

    def get_energy(self):
        pe, ke = np.zeros(self.ncells), np.zeros(self.ncells)
        self._check(lib().orc_get_energy(self._h, _p(pe), _p(ke)), "get_energy")
        return pe, ke

    def get_box(self, cell):
        H, Q, R = np.zeros((3, 3)), np.zeros((3, 3)), np.zeros((3, 3))
        J = ctypes.c_double(0)
        self._check(lib().orc_get_box(self._h, cell, _p(H), _p(Q), _p(R), ctypes.byref(J)), "get_box")
        return H, Q, R, J.value
