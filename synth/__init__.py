"""Seeded synthetic inputs: sparse coordinates, values, initial parameters.

Only random numbers live here (see ``synth.c``); none of the method's
arithmetic does.  The oracle and the GPU library both consume these arrays.

Workload recipes (the paper's datasets are not available, so these stand in
for them with the same shapes and value ranges):

* ``small``      order 3, 1000^3, 100k uniform distinct coordinates, values 1..5
* ``netflix``    order 3, 480000 x 18000 x 2200, 100M coordinates, Zipf(1.1)
                 per mode, values 1..5 (shape of the Netflix ratings tensor of
                 the experiments section, Table 2)
* ``order8``     order 8, every dim 10000, 50M coordinates, Zipf(1.05),
                 values N(3,1) clipped to [1,5] (Synthetic(Order), Table 3)
* ``order4``     order 4, 1e6 x 1e5 x 1e4 x 1e3, 200M coordinates, Zipf(1.1),
                 values 1..5
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libftsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile synth.c into libftsynth.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, u64, i32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        vp = ctypes.c_void_p
        lib.synth_coords.argtypes = [i32, vp, vp, i64, u64, vp, vp]
        lib.synth_coords.restype = i32
        lib.synth_values.argtypes = [i64, i32, dbl, dbl, dbl, dbl, u64, vp]
        lib.synth_values.restype = i32
        lib.synth_normal.argtypes = [i64, dbl, dbl, u64, u64, vp]
        lib.synth_normal.restype = i32
        lib.synth_uniform_index.argtypes = [i64, i64, u64, u64, vp]
        lib.synth_uniform_index.restype = i32
        lib.synth_draw.argtypes = [u64, u64]
        lib.synth_draw.restype = u64
        lib.synth_stream_key.argtypes = [u64, u64]
        lib.synth_stream_key.restype = u64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def coords(dims, nnz: int, zipf_s, seed: int):
    """First ``nnz`` distinct coordinates of the seeded draw sequence.

    Returns (coords int32 [order][nnz], draws_used)."""
    dims = np.ascontiguousarray(dims, dtype=np.int64)
    order = len(dims)
    if np.isscalar(zipf_s):
        zipf_s = [float(zipf_s)] * order
    zs = np.ascontiguousarray(zipf_s, dtype=np.float64)
    out = np.empty((order, int(nnz)), dtype=np.int32)
    used = np.zeros(1, dtype=np.int64)
    rc = _load().synth_coords(order, _ptr(dims), _ptr(zs), int(nnz), int(seed) & (2**64 - 1), _ptr(out), _ptr(used))
    if rc != 0:
        raise ValueError(f"synth_coords failed with status {rc}")
    return out, int(used[0])


def values(nnz: int, kind: str, seed: int):
    """Tensor values: 'int1to5' (uniform integers 1..5) or 'normal3' (N(3,1) clipped to [1,5])."""
    out = np.empty(int(nnz), dtype=np.float32)
    if kind == "int1to5":
        rc = _load().synth_values(int(nnz), 0, 1.0, 5.0, 0.0, 0.0, int(seed), _ptr(out))
    elif kind == "normal3":
        rc = _load().synth_values(int(nnz), 1, 3.0, 1.0, 1.0, 5.0, int(seed), _ptr(out))
    else:
        raise ValueError(kind)
    if rc != 0:
        raise ValueError(f"synth_values failed with status {rc}")
    return out


def normal(shape, mean: float, std: float, seed: int, tag: int) -> np.ndarray:
    out = np.empty(int(np.prod(shape)), dtype=np.float32)
    rc = _load().synth_normal(out.size, float(mean), float(std), int(seed), int(tag), _ptr(out))
    if rc != 0:
        raise ValueError(f"synth_normal failed with status {rc}")
    return out.reshape(shape)


def uniform_index(count: int, n: int, seed: int, tag: int) -> np.ndarray:
    out = np.empty(int(count), dtype=np.int32)
    rc = _load().synth_uniform_index(int(count), int(n), int(seed), int(tag), _ptr(out))
    if rc != 0:
        raise ValueError(f"synth_uniform_index failed with status {rc}")
    return out


def planted(coords_, dims, seed: int, noise: float = 0.25):
    """Values of a planted separable model, for convergence runs with a held-out test set:
    x = 1 + 4 prod_n u_n[i_n] + N(0, noise^2), clipped to [1, 5], with u_n[i] uniform in [0.3, 1)
    drawn per index of every mode.  Real structure that a low-rank model can learn, unlike the
    independent values of 'int1to5'."""
    order = len(dims)
    prod = np.ones(coords_.shape[1], dtype=np.float64)
    for n in range(order):
        u = 0.3 + 0.7 * uniform_index(int(dims[n]), 1 << 20, seed, 100 + n).astype(np.float64) / float(1 << 20)
        prod *= u[coords_[n]]
    eps = normal((coords_.shape[1],), 0.0, noise, seed, 200).astype(np.float64)
    return np.clip(1.0 + 4.0 * prod + eps, 1.0, 5.0).astype(np.float32)


def test_mask(nnz: int, seed: int, percent: int = 10):
    """Seeded held-out split: True for about `percent` % of the elements."""
    return uniform_index(int(nnz), 100, seed, 300) < percent


def init_params(dims, J, R: int, sigma: float, seed: int):
    """A(n) (I_n x J_n) and B(n) (J_n x R), entries N(0, sigma^2) rounded to float32."""
    order = len(dims)
    if np.isscalar(J):
        J = [int(J)] * order
    A = [normal((int(dims[n]), int(J[n])), 0.0, sigma, seed, 2 * n) for n in range(order)]
    B = [normal((int(J[n]), int(R)), 0.0, sigma, seed, 2 * n + 1) for n in range(order)]
    return A, B


@dataclass
class Workload:
    name: str
    dims: list
    nnz: int
    zipf: float
    value_kind: str
    J: list
    R: int
    sigma: float = 0.1
    lr: float = 1e-3
    lam: float = 1e-2
    seed: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "small": Workload("small", [1000, 1000, 1000], 100_000, 0.0, "int1to5", [8, 8, 8], 8),
    "netflix": Workload("netflix", [480_000, 18_000, 2_200], 100_000_000, 1.1, "int1to5", [16, 16, 16], 16),
    "netflix32": Workload("netflix32", [480_000, 18_000, 2_200], 100_000_000, 1.1, "int1to5", [32, 32, 32], 32),
    "order8": Workload("order8", [10_000] * 8, 50_000_000, 1.05, "normal3", [8] * 8, 16),
    "order4": Workload("order4", [1_000_000, 100_000, 10_000, 1_000], 200_000_000, 1.1, "int1to5", [32] * 4, 32),
}
# The paper's synthetic sweeps (Section 5.1 table of synthetic tensors; Sections 5.4, 5.5): uniform random
# coordinates, values 1..5, J = R = 32.  Order 3..10 with every dimension 10,000 and 100M elements; order 3
# with every dimension 1,000 and 20M..100M elements (density 2 %..10 %).
for _n in range(3, 11):
    WORKLOADS[f"sweep_order{_n}"] = Workload(f"sweep_order{_n}", [10_000] * _n, 100_000_000, 0.0, "int1to5",
                                             [32] * _n, 32)
# Convergence runs (the analogue of the paper's Figure 3): a Netflix-like shape with planted values
# and a held-out test set.
WORKLOADS["planted"] = Workload("planted", [100_000, 10_000, 1_000], 20_000_000, 1.1, "planted", [16] * 3, 16,
                                sigma=0.3, lr=1e-2, lam=1e-2)
for _m in (20, 40, 60, 80, 100):
    WORKLOADS[f"sweep_density{_m}"] = Workload(f"sweep_density{_m}", [1_000] * 3, _m * 1_000_000, 0.0, "int1to5",
                                               [32] * 3, 32)


def make(w: Workload, nnz: int | None = None, dims=None):
    """Generate (coords, vals, A, B) for a workload; ``nnz``/``dims`` override for scaled-down cases."""
    dims = list(w.dims if dims is None else dims)
    nnz = int(w.nnz if nnz is None else nnz)
    c, _ = coords(dims, nnz, w.zipf, w.seed)
    v = planted(c, dims, w.seed) if w.value_kind == "planted" else values(nnz, w.value_kind, w.seed)
    A, B = init_params(dims, w.J, w.R, w.sigma, w.seed + 1)
    return c, v, A, B
