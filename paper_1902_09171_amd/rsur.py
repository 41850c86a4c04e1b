"""Python binding of the stress-surrogate C ABI (include/rsur.h): argument marshalling only.

The surrogate lives in the same librcell.so as the MD library; every computation runs there.
Device buffers are passed as raw pointers (e.g. torch tensors' data_ptr()).
"""
import ctypes

import numpy as np

from .rcell import OK, RCellError, load as _load_lib

EXPORTS = ["rsur_create", "rsur_destroy", "rsur_last_error", "rsur_num_params", "rsur_set_params",
           "rsur_get_params", "rsur_get_grads", "rsur_set_norm", "rsur_fit_norm", "rsur_forward",
           "rsur_forward_members", "rsur_forward_static", "rsur_train_step"]

_configured = False


def load():
    global _configured
    L = _load_lib()
    if not _configured:
        vp, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
        sig = {
            "rsur_create": [i32, i32, i32, i32, i32, i32, vp, vp], "rsur_destroy": [vp],
            "rsur_last_error": [vp], "rsur_num_params": [vp, vp], "rsur_set_params": [vp, i32, vp],
            "rsur_get_params": [vp, i32, vp], "rsur_get_grads": [vp, i32, vp],
            "rsur_set_norm": [vp, vp, vp, vp, vp], "rsur_fit_norm": [vp, vp, vp, i32],
            "rsur_forward": [vp, vp, i32, vp, vp], "rsur_forward_members": [vp, vp, i32, vp],
            "rsur_forward_static": [vp, vp, i32, vp, vp],
            "rsur_train_step": [vp, vp, vp, i32, f32, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.rsur_last_error.restype = ctypes.c_char_p
        _configured = True
    return L


def _f32(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return a.reshape(shape) if shape is not None else a


class Surrogate:
    """K-member ensemble MLP (din -> depth x width -> dout) on the current GPU."""

    def __init__(self, din=153, width=256, depth=4, dout=6, ensemble=5, max_batch=4096, stream=None):
        L = load()
        h = ctypes.c_void_p()
        st = L.rsur_create(din, width, depth, dout, ensemble, max_batch, stream, ctypes.byref(h))
        if st != OK:
            raise RCellError(st, (L.rsur_last_error(None) or b"").decode())
        self._h = h
        self.din, self.width, self.depth, self.dout, self.K, self.max_batch = din, width, depth, dout, ensemble, max_batch
        n = ctypes.c_int64(0)
        self._check(L.rsur_num_params(h, ctypes.byref(n)))
        self.nparams = n.value

    def close(self):
        if getattr(self, "_h", None):
            try:
                load().rsur_destroy(self._h)
            except Exception:          # interpreter shutdown: the library is already gone
                pass
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        if st != OK:
            raise RCellError(st, (load().rsur_last_error(self._h) or b"").decode())

    @property
    def dims(self):
        return [self.din] + [self.width] * self.depth + [self.dout]

    def set_params(self, member, w):
        w = _f32(w)
        if w.size != self.nparams:                      # the library reads nparams floats
            raise ValueError(f"{w.size} parameters given, the network has {self.nparams}")
        self._check(load().rsur_set_params(self._h, member, w.ctypes.data))

    def get_params(self, member):
        w = np.zeros(self.nparams, np.float32)
        self._check(load().rsur_get_params(self._h, member, w.ctypes.data))
        return w

    def get_grads(self, member):
        g = np.zeros(self.nparams, np.float32)
        self._check(load().rsur_get_grads(self._h, member, g.ctypes.data))
        return g

    def set_norm(self, x_mu, x_sd, y_mu, y_sd):
        a = [_f32(v) for v in (x_mu, x_sd, y_mu, y_sd)]
        if [v.size for v in a] != [self.din, self.din, self.dout, self.dout]:
            raise ValueError(f"normalisation sizes {[v.size for v in a]}, expected din, din, dout, dout = "
                             f"{[self.din, self.din, self.dout, self.dout]}")
        self._check(load().rsur_set_norm(self._h, *[v.ctypes.data for v in a]))

    def fit_norm(self, X_dev_ptr, Y_dev_ptr, n):
        self._check(load().rsur_fit_norm(self._h, X_dev_ptr, Y_dev_ptr, int(n)))

    def forward(self, X_dev_ptr, B, mean_dev_ptr, var_dev_ptr=None):
        self._check(load().rsur_forward(self._h, X_dev_ptr, int(B), mean_dev_ptr, var_dev_ptr))

    def forward_static(self, X_dev_ptr, B, mean_dev_ptr, var_dev_ptr=None):
        """rsur_forward_static: the ensemble forward without any device allocation (fixed array)."""
        self._check(load().rsur_forward_static(self._h, X_dev_ptr, int(B), mean_dev_ptr, var_dev_ptr))

    def forward_members(self, X_dev_ptr, B, out_dev_ptr):
        self._check(load().rsur_forward_members(self._h, X_dev_ptr, int(B), out_dev_ptr))

    def train_step(self, X_dev_ptr, Y_dev_ptr, B, lr, want_loss=True):
        loss = np.zeros(self.K, np.float32) if want_loss else None
        self._check(load().rsur_train_step(self._h, X_dev_ptr, Y_dev_ptr, int(B), float(lr),
                                           loss.ctypes.data if want_loss else None))
        return loss
