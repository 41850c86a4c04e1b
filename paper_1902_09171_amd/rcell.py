"""Python binding of the librcell C ABI (include/rcell.h): argument marshalling only.

Every computation happens in the HIP library.  There is no fallback: if librcell.so has not
been built (``python -m paper_1902_09171_amd.build``) or cannot be loaded, importing the binding
raises.  Device memory and streams may come from PyTorch; the library itself only sees raw
pointers.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librcell.so")

OK, ERR_ARG, ERR_BAD_F, ERR_BOX, ERR_BOND, ERR_NONFINITE, ERR_OOM, ERR_DEVICE, ERR_STATE = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
POTENTIALS = {"kg": 1, "sc_eam": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}

# every entry point that include/rcell.h declares
EXPORTS = ["rcell_create", "rcell_set_deformation", "rcell_set_deformation_dev", "rcell_run",
           "rcell_get_stress", "rcell_get_stress_dev", "rcell_get_stress_ext", "rcell_destroy", "rcell_last_error",
           "rcell_get_status", "rcell_get_forces", "rcell_get_state", "rcell_set_state",
           "rcell_get_energy", "rcell_get_box", "rcell_get_rebuilds", "rcell_set_lanes",
           "rcell_get_lanes", "rcell_set_bin_factor", "rcell_get_bin_factor", "rcell_autotune", "rcell_prof_enable", "rcell_prof_read", "rcell_set_graph_steps",
           "rcell_qr_dev", "rcell_stress_return_dev", "rcell_minimize", "rcell_probe_peaks",
           "rcell_set_build_mode"]


class RCellError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"rcell error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("potential", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("dt", ctypes.c_double), ("temperature", ctypes.c_double), ("gamma", ctypes.c_double),
                ("mass", ctypes.c_double), ("kB", ctypes.c_double), ("mvv2e", ctypes.c_double),
                ("rc", ctypes.c_double), ("skin", ctypes.c_double),
                ("lj_eps", ctypes.c_double), ("lj_sigma", ctypes.c_double),
                ("fene_K", ctypes.c_double), ("fene_R0", ctypes.c_double),
                ("sc_eps", ctypes.c_double), ("sc_a", ctypes.c_double), ("sc_c", ctypes.c_double),
                ("sc_n", ctypes.c_int32), ("sc_m", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("include_kinetic", ctypes.c_int32)]


class CellInit(ctypes.Structure):
    _fields_ = [("natoms", ctypes.c_int32), ("nbonds", ctypes.c_int32),
                ("H0", ctypes.c_void_p), ("x", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("bonds", ctypes.c_void_p)]


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1902_09171_amd.build")
        # torch ships its own HIP runtime under the same soname; loading torch first lets the
        # library bind to that one, so the process holds a single HIP runtime (two copies cannot
        # share the device, and whichever initialises second reports no GPU)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        sig = {
            "rcell_create": [vp, vp, i32, vp, vp], "rcell_set_deformation": [vp, vp],
            "rcell_set_deformation_dev": [vp, vp], "rcell_run": [vp, i32],
            "rcell_minimize": [vp, i32, ctypes.c_double, vp],
            "rcell_get_stress": [vp, vp, vp], "rcell_get_stress_dev": [vp, vp, vp],
            "rcell_get_stress_ext": [vp, vp, vp, vp],
            "rcell_destroy": [vp], "rcell_last_error": [vp], "rcell_get_status": [vp, vp],
            "rcell_get_forces": [vp, i32, vp], "rcell_get_state": [vp, i32, vp, vp, vp, vp, vp],
            "rcell_set_state": [vp, i32, vp, vp, vp, vp, i64], "rcell_get_energy": [vp, vp, vp],
            "rcell_get_box": [vp, i32, vp, vp, vp, vp], "rcell_get_rebuilds": [vp, vp],
            "rcell_set_lanes": [vp, i32], "rcell_get_lanes": [vp, vp], "rcell_set_build_mode": [vp, i32],
            "rcell_set_bin_factor": [vp, i32], "rcell_get_bin_factor": [vp, vp], "rcell_autotune": [vp, i32, vp, vp],
            "rcell_prof_enable": [vp, i32], "rcell_prof_read": [vp, i32, vp, vp],
            "rcell_set_graph_steps": [vp, i32],
            "rcell_qr_dev": [vp, i32, vp, vp, vp, vp], "rcell_stress_return_dev": [vp, vp, i32, vp, vp, vp],
            "rcell_probe_peaks": [ctypes.c_size_t, vp, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.rcell_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def params_struct(p: dict) -> Params:
    s = Params()
    for name, _ in Params._fields_:
        val = p[name]
        if name == "potential" and isinstance(val, str):
            val = POTENTIALS[val]
        if name == "precision" and isinstance(val, str):
            val = PRECISIONS[val]
        setattr(s, name, val)
    return s


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a.reshape(shape) if shape is not None else a


def _p(a):
    return None if a is None else a.ctypes.data


def qr_dev(F_dev_ptr, n, Q_dev_ptr, R_dev_ptr, status_dev_ptr=None, stream=None):
    """Eq. (4) for n deformation gradients in device memory (FP64, n x 9)."""
    st = load().rcell_qr_dev(F_dev_ptr, int(n), Q_dev_ptr, R_dev_ptr, status_dev_ptr, stream)
    if st != OK:
        raise RCellError(st, "qr_dev")


def probe_peaks(copy_bytes=1 << 30, stream=None):
    """Measured copy bandwidth (GB/s, read + write) and FP32 FMA rate (TFLOP/s) of the GPU."""
    gbs, tf = ctypes.c_double(), ctypes.c_double()
    st = load().rcell_probe_peaks(int(copy_bytes), ctypes.byref(gbs), ctypes.byref(tf), stream)
    if st != OK:
        raise RCellError(st, "rcell_probe_peaks failed")
    return gbs.value, tf.value


def stress_return_dev(F_dev_ptr, sigma_md_dev_ptr, n, sigma_fem_dev_ptr, P_dev_ptr=None, stream=None):
    """Eqs. (7), (8) for n MD-frame stresses in device memory (FP64)."""
    st = load().rcell_stress_return_dev(F_dev_ptr, sigma_md_dev_ptr, int(n), sigma_fem_dev_ptr, P_dev_ptr, stream)
    if st != OK:
        raise RCellError(st, "stress_return_dev")


class RCellBatch:
    """A batch of r-cells on the current GPU (one rcell_ctx).

    params: dict with the rcell_params fields; cells: list of {"x", "v", "bonds", "H0"}.
    stream: optional hipStream_t handle (int), e.g. torch.cuda.current_stream().cuda_stream.
    """

    def __init__(self, params, cells, stream=None):
        L = load()
        self.params = dict(params)
        self.ncells = len(cells)
        self.natoms = [len(c["x"]) for c in cells]
        self._keep = []
        inits = (CellInit * self.ncells)()
        for k, c in enumerate(cells):
            H0 = _f64(c["H0"], (3, 3))
            x = _f64(c["x"], (-1, 3))
            v = None if c.get("v") is None else _f64(c["v"], (-1, 3))
            if v is not None and v.shape != x.shape:     # the library reads natoms rows of each
                raise ValueError(f"cell {k}: v has shape {v.shape}, x has {x.shape}")
            b = np.ascontiguousarray(np.asarray(c.get("bonds", np.zeros((0, 2))), np.int32).reshape(-1, 2))
            self._keep += [H0, x, v, b]
            inits[k].natoms = len(x)
            inits[k].nbonds = len(b)
            inits[k].H0 = _p(H0)
            inits[k].x = _p(x)
            inits[k].v = _p(v)
            inits[k].bonds = _p(b) if len(b) else None
        ps = params_struct(params)
        h = ctypes.c_void_p()
        st = L.rcell_create(ctypes.byref(ps), inits, self.ncells, stream, ctypes.byref(h))
        self._keep = []
        if st != OK:
            raise RCellError(st, (L.rcell_last_error(None) or b"").decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().rcell_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        if st != OK:
            raise RCellError(st, (load().rcell_last_error(self._h) or b"").decode())

    def set_deformation(self, F):
        F = _f64(F, (self.ncells, 3, 3))
        self._check(load().rcell_set_deformation(self._h, _p(F)))

    def set_deformation_dev(self, F_dev_ptr):
        self._check(load().rcell_set_deformation_dev(self._h, F_dev_ptr))

    def run(self, nsteps):
        self._check(load().rcell_run(self._h, int(nsteps)))

    def minimize(self, max_iter, ftol):
        """Molecular statics (FIRE relaxation in the current boxes); returns the moves per cell."""
        iters = np.zeros(self.ncells, np.int32)
        self._check(load().rcell_minimize(self._h, int(max_iter), float(ftol), iters.ctypes.data))
        return iters

    def get_stress(self, with_P=False):
        s = np.zeros((self.ncells, 6))
        P = np.zeros((self.ncells, 3, 3)) if with_P else None
        self._check(load().rcell_get_stress(self._h, _p(s), _p(P)))
        return (s, P) if with_P else s

    def get_stress_ext(self):
        """(sigma_FEM, P, sigma_MD) of the window, clearing it."""
        s, P, smd = np.zeros((self.ncells, 6)), np.zeros((self.ncells, 3, 3)), np.zeros((self.ncells, 6))
        self._check(load().rcell_get_stress_ext(self._h, _p(s), _p(P), _p(smd)))
        return s, P, smd

    def get_stress_dev(self, sigma_dev_ptr, P_dev_ptr=None):
        self._check(load().rcell_get_stress_dev(self._h, sigma_dev_ptr, P_dev_ptr))

    def status(self):
        s = np.zeros(self.ncells, np.int32)
        self._check(load().rcell_get_status(self._h, _p(s)))
        return s

    def get_forces(self, cell):
        f = np.zeros((self.natoms[cell], 3))
        self._check(load().rcell_get_forces(self._h, cell, _p(f)))
        return f

    def get_state(self, cell):
        n = self.natoms[cell]
        x, v, H, Rp = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((3, 3)), np.zeros((3, 3))
        step = ctypes.c_int64(0)
        self._check(load().rcell_get_state(self._h, cell, _p(x), _p(v), _p(H), _p(Rp), ctypes.byref(step)))
        return dict(x=x, v=v, H=H, Rprev=Rp, step=step.value)

    def set_state(self, cell, x, v, H, Rprev, step):
        if not 0 <= cell < self.ncells:
            raise IndexError(f"cell {cell} of {self.ncells}")
        x, v, H, Rp = _f64(x, (-1, 3)), _f64(v, (-1, 3)), _f64(H, (3, 3)), _f64(Rprev, (3, 3))
        n = self.natoms[cell]
        if x.shape != (n, 3) or v.shape != (n, 3):       # the library reads n rows of each
            raise ValueError(f"cell {cell} has {n} atoms: x {x.shape}, v {v.shape}")
        self._check(load().rcell_set_state(self._h, cell, _p(x), _p(v), _p(H), _p(Rp), int(step)))

    def get_energy(self):
        pe, ke = np.zeros(self.ncells), np.zeros(self.ncells)
        self._check(load().rcell_get_energy(self._h, _p(pe), _p(ke)))
        return pe, ke

    def get_box(self, cell):
        H, Q, R = np.zeros((3, 3)), np.zeros((3, 3)), np.zeros((3, 3))
        J = ctypes.c_double(0)
        self._check(load().rcell_get_box(self._h, cell, _p(H), _p(Q), _p(R), ctypes.byref(J)))
        return H, Q, R, J.value

    def rebuilds(self):
        c = ctypes.c_int64(0)
        self._check(load().rcell_get_rebuilds(self._h, ctypes.byref(c)))
        return c.value

    def set_lanes(self, lanes):
        self._check(load().rcell_set_lanes(self._h, int(lanes)))
        return self.lanes()

    def set_bin_factor(self, f):
        """Neighbour bins at least (rc + skin) / f wide (f = 1 or 2), from each cell's next build."""
        self._check(load().rcell_set_bin_factor(self._h, int(f)))

    def bin_factor(self):
        f = ctypes.c_int32(0)
        self._check(load().rcell_get_bin_factor(self._h, ctypes.byref(f)))
        return f.value

    def autotune(self, use_cache=True):
        """Bin factor and lanes per atom timed on this batch (the state is left as found); returns
        (lanes, bin_factor)."""
        l, f = ctypes.c_int32(0), ctypes.c_int32(0)
        self._check(load().rcell_autotune(self._h, 1 if use_cache else 0, ctypes.byref(l), ctypes.byref(f)))
        return l.value, f.value

    def set_build_mode(self, mode):
        """0: automatic, 1: one block per cell for the rebuild preparation, 2: phase kernels."""
        self._check(load().rcell_set_build_mode(self._h, int(mode)))

    def set_graph_steps(self, steps):
        self._check(load().rcell_set_graph_steps(self._h, int(steps)))

    def prof_enable(self, on=True):
        self._check(load().rcell_prof_enable(self._h, 1 if on else 0))

    def prof_read(self, which=0):
        """(total_ms, launches) of pass `which` (0 force, 1 EAM density) since the last read."""
        ms, n = ctypes.c_double(0), ctypes.c_int64(0)
        self._check(load().rcell_prof_read(self._h, int(which), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def lanes(self):
        l = ctypes.c_int32(0)
        self._check(load().rcell_get_lanes(self._h, ctypes.byref(l)))
        return l.value
