"""Kremer-Grest bead-spring melt inputs (Sec. 3.2 uses standard KG chains at number density 0.85).

Chains are random walks with bond length 0.97 sigma grown with soft excluded-volume rejection in
a cubic box of edge (N/0.85)^(1/3).  The native walker lives in csrc/kgwalk.c and is compiled with
gcc on first use.  These states are not equilibrated melts; they stand in for them.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "kgwalk.c")
_LIB = os.path.join(_HERE, "_kgwalk.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.kg_random_walk.restype = ctypes.c_int
        lib.kg_random_walk.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                       ctypes.c_uint64, ctypes.c_void_p]
        lib.kg_relax.restype = ctypes.c_double
        lib.kg_relax.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                 ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int32]
        _lib = lib
    return _lib


def kg_box_edge(n: int, density: float = 0.85) -> float:
    return (n / density) ** (1.0 / 3.0)


def kg_melt(chain_lengths, seed: int, density: float = 0.85, bond: float = 0.97,
            dmin: float = 0.85, ntries: int = 200, dpush: float = 0.9, relax_iters: int = 60):
    """Return (x [N,3] in [0,L)^3, bonds [Nb,2] int32, H0 [3,3]) for the given chain lengths.

    After the walk, a geometric relaxation pushes non-bonded beads closer than dpush apart and
    restores bond lengths (see kg_relax in csrc/kgwalk.c)."""
    lens = np.ascontiguousarray(np.asarray(chain_lengths, dtype=np.int32))
    n = int(lens.sum())
    L = kg_box_edge(n, density)
    x = np.zeros((n, 3), dtype=np.float64)
    rc = _load().kg_random_walk(L, len(lens), lens.ctypes.data, bond, dmin, ntries,
                                seed & ((1 << 64) - 1), x.ctypes.data)
    if rc != 0:
        raise RuntimeError("kg_random_walk failed")
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    bonds = [np.stack([s + np.arange(l - 1), s + np.arange(1, l)], axis=1)
             for s, l in zip(starts, lens) if l > 1]
    bonds = np.ascontiguousarray((np.concatenate(bonds) if bonds else np.zeros((0, 2))).astype(np.int32))
    if relax_iters > 0 and n > 1:
        _load().kg_relax(L, n, x.ctypes.data, len(bonds), bonds.ctypes.data if len(bonds) else None,
                         dpush, bond, relax_iters)
    return x, bonds, np.eye(3) * L
