"""FP64 CPU oracle of sparse FasterTucker (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it,
and it shares no code with the GPU path: both consume the same seeded input
arrays and nothing else.

The arithmetic lives in ``ft_oracle.c`` (plain C loops in FP64); this module
only marshals numpy arrays.  Each method names the passage of the paper it
follows; the readings of ambiguous passages are listed in the C file header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ft_oracle.c")
# FT_ORACLE_LIB points the loader at another build of ft_oracle.c (the pin-sensitivity test loads copies
# with planted mistakes); build() always writes the default path
_DEFAULT_LIB = os.path.join(_HERE, "libftoracle.so")
_LIB = os.environ.get("FT_ORACLE_LIB") or _DEFAULT_LIB
_lib = None


def build(force: bool = True) -> str:
    """Compile ft_oracle.c (gcc -O2, no fast-math, single-threaded)."""
    if force or not os.path.exists(_DEFAULT_LIB):
        tmp = _DEFAULT_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _DEFAULT_LIB)
    return _DEFAULT_LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            if _LIB != _DEFAULT_LIB:
                raise FileNotFoundError(_LIB)
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        lib.orc_refresh.argtypes = [i64, i32, i32, vp, vp, vp]
        lib.orc_refresh.restype = None
        lib.orc_predict.argtypes = [i32, i32, vp, vp, i64, i64, vp]
        lib.orc_predict.restype = None
        lib.orc_factor_pass.argtypes = [i32, vp, vp, i32, vp, vp, vp, vp, vp, i64, i32, dbl, dbl]
        lib.orc_factor_pass.restype = i32
        lib.orc_factor_pass_relaxed.argtypes = [i32, vp, vp, i32, vp, vp, vp, vp, vp, i64, i32, dbl, dbl, i64, i64]
        lib.orc_factor_pass_relaxed.restype = i32
        lib.orc_core_grad.argtypes = [i32, vp, i32, vp, vp, vp, vp, vp, i64, i32, vp]
        lib.orc_core_grad.restype = i32
        lib.orc_core_pass.argtypes = [i32, vp, i32, vp, vp, vp, vp, vp, i64, i32, dbl, dbl]
        lib.orc_core_pass.restype = i32
        lib.orc_epoch.argtypes = [i32, vp, vp, i32, vp, vp, vp, vp, vp, i64, dbl, dbl, dbl, dbl]
        lib.orc_epoch.restype = i32
        lib.orc_loss.argtypes = [i32, vp, vp, i32, vp, vp, vp, vp, vp, i64, dbl, dbl, vp]
        lib.orc_loss.restype = None
        lib.orc_grad.argtypes = [i32, vp, vp, i32, vp, vp, vp, vp, vp, i64, vp, vp, vp]
        lib.orc_grad.restype = i32
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _parr(arrs):
    t = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    return t


class Model:
    """Parameters A(n), B(n), cached C(n) = A(n) B(n) and one sparse tensor, all FP64."""

    def __init__(self, dims, J, R, coords, vals, A, B):
        self.N = len(dims)
        self.dims = np.ascontiguousarray(dims, dtype=np.int64)
        Jl = [int(J)] * self.N if np.isscalar(J) else [int(j) for j in J]
        self.J = np.ascontiguousarray(Jl, dtype=np.int32)
        self.R = int(R)
        self.coords = np.ascontiguousarray(coords, dtype=np.int32)
        self.nnz = int(self.coords.shape[1])
        self.vals = np.ascontiguousarray(vals, dtype=np.float64)
        self.A = [np.ascontiguousarray(a, dtype=np.float64).copy() for a in A]
        self.B = [np.ascontiguousarray(b, dtype=np.float64).copy() for b in B]
        self.C = [np.zeros((int(self.dims[n]), self.R)) for n in range(self.N)]
        self.refresh()

    def _common(self):
        return (self.N, _p(self.dims), _p(self.J), self.R)

    def refresh(self, m=None):
        """C(n) = A(n) B(n) (Section 3.1)."""
        modes = range(self.N) if m is None else [m]
        for n in modes:
            _load().orc_refresh(int(self.dims[n]), int(self.J[n]), self.R, _p(self.A[n]), _p(self.B[n]), _p(self.C[n]))

    def predict(self, coords) -> np.ndarray:
        """xhat = sum_r prod_n C(n)[i_n, r] (Eq. (1) via Eq. (12))."""
        c = np.ascontiguousarray(coords, dtype=np.int32)
        q = c.shape[1]
        out = np.empty(q)
        _load().orc_predict(self.N, self.R, _parr(self.C), _p(c), q, q, _p(out))
        return out

    def factor_pass(self, m, lr, lam):
        """Factor module of Algorithm 2 for mode m (no refresh of C(m))."""
        rc = _load().orc_factor_pass(*self._common(), _parr(self.A), _parr(self.B), _parr(self.C), _p(self.coords),
                                     _p(self.vals), self.nnz, int(m), float(lr), float(lam))
        if rc:
            raise RuntimeError(f"orc_factor_pass: {rc}")

    def factor_pass_relaxed(self, m, lr, lam, head, chunk):
        """Relaxed factor module for mode m (the chunks of a long row all read the row as its head left it,
        as concurrent workers of Algorithm 4 would; their increments are merged under a step guard).  No
        refresh of C(m).  The reading is stated in ft_oracle.c."""
        rc = _load().orc_factor_pass_relaxed(*self._common(), _parr(self.A), _parr(self.B), _parr(self.C),
                                             _p(self.coords), _p(self.vals), self.nnz, int(m), float(lr), float(lam),
                                             int(head), int(chunk))
        if rc:
            raise RuntimeError(f"orc_factor_pass_relaxed: {rc}")

    def epoch_relaxed(self, lr_a, lam_a, lr_b, lam_b, head, chunk):
        """One iteration of Algorithm 2 with the relaxed factor module."""
        for m in range(self.N):
            self.factor_pass_relaxed(m, lr_a, lam_a, head, chunk)
            self.refresh(m)
        for m in range(self.N):
            self.core_pass(m, lr_b, lam_b)
            self.refresh(m)

    def core_grad(self, m) -> np.ndarray:
        """G = sum_x e_x a_{i_m} w_x^T over Omega (Eq. (11), Algorithm 5)."""
        G = np.zeros((int(self.J[m]), self.R))
        rc = _load().orc_core_grad(self.N, _p(self.J), self.R, _parr(self.A), _parr(self.B), _parr(self.C),
                                   _p(self.coords), _p(self.vals), self.nnz, int(m), _p(G))
        if rc:
            raise RuntimeError(f"orc_core_grad: {rc}")
        return G

    def core_pass(self, m, lr, lam):
        """Core module of Algorithm 2 for mode m (no refresh of C(m))."""
        rc = _load().orc_core_pass(self.N, _p(self.J), self.R, _parr(self.A), _parr(self.B), _parr(self.C),
                                   _p(self.coords), _p(self.vals), self.nnz, int(m), float(lr), float(lam))
        if rc:
            raise RuntimeError(f"orc_core_pass: {rc}")

    def epoch(self, lr_a, lam_a, lr_b, lam_b):
        """One iteration of Algorithm 2 (factor module, then core module)."""
        rc = _load().orc_epoch(*self._common(), _parr(self.A), _parr(self.B), _parr(self.C), _p(self.coords),
                               _p(self.vals), self.nnz, float(lr_a), float(lam_a), float(lr_b), float(lam_b))
        if rc:
            raise RuntimeError(f"orc_epoch: {rc}")

    def loss(self, lam_a=0.0, lam_b=0.0) -> np.ndarray:
        """[SSE, RMSE, sum lam_a ||A||^2, sum lam_b ||B||^2] (Eq. (6))."""
        out = np.zeros(4)
        _load().orc_loss(*self._common(), _parr(self.A), _parr(self.B), _parr(self.C), _p(self.coords),
                         _p(self.vals), self.nnz, float(lam_a), float(lam_b), _p(out))
        return out

    def grad(self, upstream=None):
        """dL/dA(n), dL/dB(n) for dL/dxhat = upstream (None: -(x - xhat))."""
        gA = [np.zeros_like(a) for a in self.A]
        gB = [np.zeros_like(b) for b in self.B]
        up = None if upstream is None else np.ascontiguousarray(upstream, dtype=np.float64)
        rc = _load().orc_grad(*self._common(), _parr(self.A), _parr(self.B), _parr(self.C), _p(self.coords),
                              _p(self.vals), self.nnz, None if up is None else _p(up), _parr(gA), _parr(gB))
        if rc:
            raise RuntimeError(f"orc_grad: {rc}")
        return gA, gB
