"""ctypes binding of the warm-start network (include/dd_mlp.h).

Argument marshalling only: the forward pass, the gradients and the Adam steps
run in the library's kernels (BF16 matrix cores, FP32 accumulation).  Device
arrays are torch CUDA tensors; host arrays are numpy.
"""
import ctypes as C

import numpy as np

from . import dd

lib = dd.lib
_P = C.POINTER
lib.dd_mlp_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_ulonglong, C.c_void_p,
                              _P(C.c_void_p)]
lib.dd_mlp_free.argtypes = [C.c_void_p]
lib.dd_mlp_free.restype = None
lib.dd_mlp_last_error.argtypes = [C.c_void_p]
lib.dd_mlp_last_error.restype = C.c_char_p
lib.dd_mlp_shape.argtypes = [C.c_void_p, _P(C.c_int), _P(C.c_int), _P(C.c_int), _P(C.c_size_t)]
lib.dd_mlp_set_params.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
lib.dd_mlp_get_params.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
lib.dd_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
lib.dd_mlp_forward_bf16.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
lib.dd_mlp_loss_grad.argtypes = [C.c_void_p] + [C.c_void_p] * 3 + [C.c_int, _P(C.c_float),
                                                                  C.c_void_p]
lib.dd_mlp_train_step.argtypes = [C.c_void_p] + [C.c_void_p] * 3 + [C.c_int, C.c_float,
                                                                   _P(C.c_float)]
for _n in ("dd_mlp_create", "dd_mlp_shape", "dd_mlp_set_params", "dd_mlp_get_params",
           "dd_mlp_forward", "dd_mlp_forward_bf16", "dd_mlp_loss_grad", "dd_mlp_train_step"):
    getattr(lib, _n).restype = C.c_int


def _dev(t):
    import torch
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


class MLP:
    """n_in -> width -> width -> width -> n_out perceptron on the GPU."""

    def __init__(self, n_in, n_out=64, width=256, seed=0, stream=None):
        h = C.c_void_p()
        rc = lib.dd_mlp_create(n_in, n_out, width, seed, stream, C.byref(h))
        if rc != 0:
            raise ValueError(f"dd_mlp_create failed ({rc})")
        self._h = h
        a, b, c, n = C.c_int(), C.c_int(), C.c_int(), C.c_size_t()
        lib.dd_mlp_shape(h, C.byref(a), C.byref(b), C.byref(c), C.byref(n))
        self.n_in, self.n_out, self.width, self.n_params = a.value, b.value, c.value, n.value
        self.dims = [self.n_in, self.width, self.width, self.width, self.n_out]

    @property
    def handle(self):
        return self._h

    def _chk(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} failed ({rc}): {lib.dd_mlp_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None) and lib is not None:
            lib.dd_mlp_free(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        self._chk(lib.dd_mlp_get_params(self._h, out.ctypes.data_as(C.c_void_p), self.n_params),
                  "dd_mlp_get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params
        self._chk(lib.dd_mlp_set_params(self._h, p.ctypes.data_as(C.c_void_p), p.size),
                  "dd_mlp_set_params")

    def forward(self, x):
        import torch
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device=x.device)
        self._chk(lib.dd_mlp_forward(self._h, _dev(x), x.shape[0], _dev(y)), "dd_mlp_forward")
        return y

    def loss_grad(self, x, t, mask):
        loss = C.c_float()
        g = np.empty(self.n_params, dtype=np.float32)
        self._chk(lib.dd_mlp_loss_grad(self._h, _dev(x), _dev(t), _dev(mask), x.shape[0],
                                       C.byref(loss), g.ctypes.data_as(C.c_void_p)),
                  "dd_mlp_loss_grad")
        return loss.value, g

    def train_step(self, x, t, mask, lr):
        loss = C.c_float()
        self._chk(lib.dd_mlp_train_step(self._h, _dev(x), _dev(t), _dev(mask), x.shape[0],
                                        float(lr), C.byref(loss)), "dd_mlp_train_step")
        return loss.value
