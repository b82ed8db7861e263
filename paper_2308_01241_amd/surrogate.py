"""Python handle over the surrogate MLP and top-k of the C ABI (argument
marshalling only; the products run on MFMA in the library's kernels)."""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import check, load


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class MLP:
    def __init__(self, n_in=100, hidden=256, n_hidden=3, n_out=40, seed=0, stream=None):
        lib = load()
        self._lib = lib
        h = ctypes.c_void_p()
        s = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        check(lib.dtb_mlp_create(n_in, hidden, n_hidden, n_out, int(seed), s, ctypes.byref(h)))
        self._h = h
        self.n_in, self.n_out = n_in, n_out
        self.shapes = [(d1, d0) for d0, d1 in zip([n_in] + [hidden] * n_hidden, [hidden] * n_hidden + [n_out])]
        self.num_params = int(lib.dtb_mlp_num_params(h))

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.dtb_mlp_destroy(h)
        self._h = None

    def __del__(self):
        self.close()

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.num_params, dtype=np.float32)
        check(self._lib.dtb_mlp_params(self._h, _ptr(out), 1, 0))
        return out

    def set_params(self, theta) -> None:
        t = _f32(theta)
        assert t.size == self.num_params
        check(self._lib.dtb_mlp_params(self._h, _ptr(t), 0, 0))

    def set_operands(self, fp32: bool) -> None:
        """FP32 matrix operands (True) or bfloat16 (False, the default)."""
        check(self._lib.dtb_mlp_set_operands(self._h, 1 if fp32 else 0))

    def forward(self, X) -> np.ndarray:
        X = _f32(X).reshape(-1, self.n_in)
        Y = np.zeros((X.shape[0], self.n_out), dtype=np.float32)
        check(self._lib.dtb_mlp_forward(self._h, _ptr(X), X.shape[0], _ptr(Y), 0))
        return Y

    def grad(self, X, T):
        X = _f32(X).reshape(-1, self.n_in)
        T = _f32(T).reshape(-1, self.n_out)
        g = np.zeros(self.num_params, dtype=np.float32)
        loss = ctypes.c_float(0)
        check(self._lib.dtb_mlp_grad(self._h, _ptr(X), _ptr(T), X.shape[0], ctypes.byref(loss), _ptr(g), 0))
        return float(loss.value), g

    def train_step(self, X, T, lr: float) -> float:
        X = _f32(X).reshape(-1, self.n_in)
        T = _f32(T).reshape(-1, self.n_out)
        loss = ctypes.c_float(0)
        check(self._lib.dtb_mlp_train_step(self._h, _ptr(X), _ptr(T), X.shape[0], float(lr), ctypes.byref(loss), 0))
        return float(loss.value)


def topk(scores, k: int) -> np.ndarray:
    """Indices of the k smallest scores (ties by index), via the library."""
    lib = load()
    s = _f32(scores).ravel()
    idx = np.zeros(k, dtype=np.int32)
    check(lib.dtb_topk(_ptr(s), s.size, int(k), _ptr(idx), None, 0))
    return idx


def topk_noalloc(scores, k: int, stream=None) -> np.ndarray:
    """topk through the entry point that allocates no device memory (its
    scores and indices pass through the library's static staging area)."""
    lib = load()
    s = _f32(scores).ravel()
    idx = np.zeros(k, dtype=np.int32)
    h = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    check(lib.dtb_topk_noalloc(_ptr(s), s.size, int(k), _ptr(idx), h))
    return idx
