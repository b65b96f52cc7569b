"""Python names for the C-ABI calls (argument marshalling only).

Every function takes a :class:`Plan` (the sorted sparse tensor, built once)
and a :class:`Params` (device tensors A(n), B(n), C(n) and the parameter
set's scratch) and enqueues its kernels on torch's current stream.  Nothing
here computes on the host.  torch allocates every device buffer the library
uses: the plan's workspace and each parameter set's scratch, sized by
ft_plan_query.  Shapes, dtypes and devices of the tensors are checked here
before any library call, so a mismatched tensor raises instead of reaching a
kernel.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import FtDesc, FtModeInfo, FtParams, check, load


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def supported(order: int, J: int, R: int) -> bool:
    return bool(load().ft_supported(order, J, R))


def _bytes_tensor(nbytes: int, device):
    """A device buffer of at least nbytes (torch allocations are 256-byte aligned)."""
    import torch

    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Plan:
    """Per-mode sorted copies of one sparse tensor plus work lists (ft_plan_create / ft_plan_upload).

    coords: int32 [order][nnz] (host), vals: float32 [nnz] (host).  The device arrays live in
    `self.workspace`, a torch tensor of `device_bytes` bytes owned by this object."""

    def __init__(self, dims, J, R, coords, vals, chunk=0, fanin=0, keep_host=False, with_perm=False, upload=True,
                 fiber_share=True, head=0, c_cache=True, relaxed=False, fused=True, run_reuse=False, device="cuda"):
        lib = load()
        coords = np.ascontiguousarray(coords, dtype=np.int32)
        vals = np.ascontiguousarray(vals, dtype=np.float32)
        order = len(dims)
        if coords.ndim != 2 or coords.shape[0] != order or vals.shape != (coords.shape[1],):
            raise ValueError("coords must be [order][nnz] and vals [nnz]")
        Js = [int(J)] * order if np.isscalar(J) else [int(j) for j in J]
        d = FtDesc()
        d.order = order
        for n in range(order):
            d.dims[n] = int(dims[n])
            d.J[n] = Js[n]
        d.R = int(R)
        d.nnz = int(coords.shape[1])
        d.chunk = int(chunk)
        d.head = int(head)
        d.fanin = int(fanin)
        d.flags = ((_lib.FT_KEEP_HOST if keep_host else 0) | (_lib.FT_WITH_PERM if with_perm else 0)
                   | (0 if fiber_share else _lib.FT_NO_FIBER_SHARE) | (0 if c_cache else _lib.FT_NO_C_CACHE)
                   | (_lib.FT_RELAXED if relaxed else 0) | (0 if fused else _lib.FT_SPLIT_FACTOR)
                   | (_lib.FT_RUN_REUSE if run_reuse else 0))
        self.dims = [int(x) for x in dims]
        self.order = order
        self.J = Js[0]
        self.R = int(R)
        self.nnz = int(coords.shape[1])
        self.with_perm = bool(with_perm)
        self.device = device
        self.workspace = None
        self._lib = lib
        self._h = ctypes.c_void_p()
        check(lib.ft_plan_create(ctypes.byref(self._h), ctypes.byref(d), coords.ctypes.data, vals.ctypes.data))
        dev_b, scr_b = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib.ft_plan_query(self._h, ctypes.byref(dev_b), ctypes.byref(scr_b)))
        self.device_bytes = int(dev_b.value)
        self.scratch_bytes = int(scr_b.value)
        if upload:
            self.upload()

    def upload(self):
        """Allocate the workspace (torch) and copy the plan into it on the current stream."""
        ws = _bytes_tensor(self.device_bytes, self.device)
        check(self._lib.ft_plan_upload(self._h, ws.data_ptr(), ws.numel(), _stream()))
        self.workspace = ws

    @property
    def handle(self):
        return self._h

    def mode_info(self, m: int) -> dict:
        info = FtModeInfo()
        check(self._lib.ft_plan_mode_info(self._h, int(m), ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in FtModeInfo._fields_}

    def host_csr(self, m: int, factor_order: bool = False):
        """(row_ptr, idx [(N-1), nnz], vals, perm) of mode m (plan built with keep_host=True); with factor_order,
        in the order the factor passes read (long rows dealt under relaxed=True)."""
        I = self.dims[m]
        row_ptr = np.empty(I + 1, dtype=np.int64)
        idx = np.empty((self.order - 1, self.nnz), dtype=np.int32)
        vals = np.empty(self.nnz, dtype=np.float32)
        perm = np.empty(self.nnz, dtype=np.int64)
        check(self._lib.ft_plan_host_csr(self._h, int(m), 1 if factor_order else 0, row_ptr.ctypes.data,
                                         idx.ctypes.data, vals.ctypes.data, perm.ctypes.data))
        return row_ptr, idx, vals, perm

    def profile(self, enable: bool = True):
        """Start (or stop) per-kernel event timing on this plan; clears the counters."""
        check(self._lib.ft_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{kernel: (total ms, launches)} since the last read; waits for the recorded events."""
        ms = np.zeros(len(_lib.KERNELS), dtype=np.float64)
        cnt = np.zeros(len(_lib.KERNELS), dtype=np.int64)
        check(self._lib.ft_profile_read(self._h, ms.ctypes.data, cnt.ctypes.data))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(_lib.KERNELS)}

    def close(self):
        if self._h is not None and self._h.value:
            self._lib.ft_plan_destroy(self._h)
            self._h = ctypes.c_void_p()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Params:
    """Device parameters as contiguous CUDA tensors.

    storage "f32": A(n) (I_n x J), B(n) (J x R), C(n) (I_n x R), float32.
    storage "bf16": float32 masters A(n), B(n) plus bfloat16 copies A16, B16 and C16 (C is not used).
    `scratch` is the parameter set's scratch buffer; the calls below (re)allocate it through torch
    when a plan needs more than it holds."""

    def __init__(self, A, B, C=None, device="cuda", storage="f32"):
        import torch

        if storage not in ("f32", "bf16"):
            raise ValueError("storage must be 'f32' or 'bf16'")
        self.storage = storage
        self.A = [torch.as_tensor(a, dtype=torch.float32).to(device).contiguous() for a in A]
        self.B = [torch.as_tensor(b, dtype=torch.float32).to(device).contiguous() for b in B]
        self.A16 = self.B16 = self.C16 = None
        if storage == "bf16":
            self.A16 = [torch.empty(a.shape, dtype=torch.bfloat16, device=device) for a in self.A]
            self.B16 = [torch.empty(b.shape, dtype=torch.bfloat16, device=device) for b in self.B]
            self.C16 = [torch.empty((a.shape[0], b.shape[1]), dtype=torch.bfloat16, device=device)
                        for a, b in zip(self.A, self.B)]
            self.C = [None] * len(self.A)
        elif C is None:
            self.C = [torch.empty((a.shape[0], b.shape[1]), dtype=torch.float32, device=device)
                      for a, b in zip(self.A, self.B)]
        else:
            self.C = list(C)
        self.scratch = None

    def ensure_scratch(self, nbytes: int):
        if self.scratch is None or self.scratch.numel() < nbytes:
            self.scratch = _bytes_tensor(nbytes, self.A[0].device)
        return self.scratch

    def check(self, plan: "Plan"):
        """Raise ValueError unless every tensor has the shape, dtype and placement the plan's kernels assume."""
        import torch

        N = plan.order
        if len(self.A) != N or len(self.B) != N or len(self.C) != N:
            raise ValueError(f"expected {N} matrices A, B and C, got {len(self.A)}, {len(self.B)}, {len(self.C)}")

        def want(t, name, shape, dtype):
            if t is None:
                raise ValueError(f"{name} is missing")
            if not isinstance(t, torch.Tensor) or not t.is_cuda:
                raise ValueError(f"{name} must be a CUDA tensor")
            if tuple(t.shape) != tuple(shape) or t.dtype != dtype:
                raise ValueError(f"{name} must be {dtype} of shape {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")
            if not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous")

        J, R = plan.J, plan.R
        for n in range(N):
            I = plan.dims[n]
            want(self.A[n], f"A[{n}]", (I, J), torch.float32)
            want(self.B[n], f"B[{n}]", (J, R), torch.float32)
            if self.storage == "f32":
                want(self.C[n], f"C[{n}]", (I, R), torch.float32)
            else:
                want(self.A16[n], f"A16[{n}]", (I, J), torch.bfloat16)
                want(self.B16[n], f"B16[{n}]", (J, R), torch.bfloat16)
                want(self.C16[n], f"C16[{n}]", (I, R), torch.bfloat16)

    def struct(self, plan: "Plan", with_scratch: bool = True) -> FtParams:
        """The ft_params of this set for calls with `plan` (validated; scratch sized for the plan, or none with
        with_scratch=False for the entry points that use no caller scratch)."""
        self.check(plan)
        scratch = self.ensure_scratch(plan.scratch_bytes) if with_scratch else None
        s = FtParams()
        s.storage = _lib.FT_STORE_BF16 if self.storage == "bf16" else _lib.FT_STORE_F32
        for n in range(len(self.A)):
            s.A[n] = self.A[n].data_ptr()
            s.B[n] = self.B[n].data_ptr()
            if self.storage == "f32":
                s.C[n] = self.C[n].data_ptr()
            else:
                s.A16[n] = self.A16[n].data_ptr()
                s.B16[n] = self.B16[n].data_ptr()
                s.C16[n] = self.C16[n].data_ptr()
        s.scratch = scratch.data_ptr() if scratch is not None else None
        s.scratch_bytes = scratch.numel() if scratch is not None else 0
        return s

    def clone(self) -> "Params":
        p = Params.__new__(Params)
        p.storage = self.storage
        p.A = [a.clone() for a in self.A]
        p.B = [b.clone() for b in self.B]
        p.C = [None if c is None else c.clone() for c in self.C]
        p.A16 = None if self.A16 is None else [t.clone() for t in self.A16]
        p.B16 = None if self.B16 is None else [t.clone() for t in self.B16]
        p.C16 = None if self.C16 is None else [t.clone() for t in self.C16]
        p.scratch = None
        return p


def _p(plan: Plan, params: Params):
    if plan.workspace is None:
        raise RuntimeError("plan not uploaded")
    return ctypes.byref(params.struct(plan))


def _device_vector(t, name, n, dtype):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or t.numel() != n \
            or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor of {n} elements")


def refresh(plan: Plan, params: Params, mode: int = -1):
    check(plan._lib.ft_refresh(plan.handle, _p(plan, params), int(mode), _stream()))


def predict(plan: Plan, params: Params, coords):
    """coords: int32 CUDA tensor [order][q] -> float32 CUDA tensor [q].

    The indices are checked against the dimensions here (the kernel gathers them unchecked)."""
    import torch

    if not isinstance(coords, torch.Tensor) or not coords.is_cuda or coords.dtype != torch.int32 \
            or coords.dim() != 2 or coords.shape[0] != plan.order:
        raise ValueError(f"coords must be an int32 CUDA tensor of shape [{plan.order}][q]")
    coords = coords.contiguous()
    q = coords.shape[1]
    if q > 0:
        lo = coords.amin(dim=1).cpu().numpy()
        hi = coords.amax(dim=1).cpu().numpy()
        for n in range(plan.order):
            if lo[n] < 0 or hi[n] >= plan.dims[n]:
                raise ValueError(f"coordinate of mode {n} out of range [0, {plan.dims[n]})")
    out = torch.empty(q, dtype=torch.float32, device=coords.device)
    check(plan._lib.ft_predict(plan.handle, _p(plan, params), coords.data_ptr(), q, out.data_ptr(), _stream()))
    return out


def factor_pass(plan: Plan, params: Params, mode: int, lr: float, lam: float):
    check(plan._lib.ft_factor_pass(plan.handle, _p(plan, params), int(mode), float(lr), float(lam), _stream()))


def factor_epoch(plan: Plan, params: Params, lr: float, lam: float):
    check(plan._lib.ft_factor_epoch(plan.handle, _p(plan, params), float(lr), float(lam), _stream()))


def core_grad(plan: Plan, params: Params, mode: int):
    import torch

    G = torch.empty((plan.J, plan.R), dtype=torch.float32, device=params.A[0].device)
    check(plan._lib.ft_core_grad(plan.handle, _p(plan, params), int(mode), G.data_ptr(), _stream()))
    return G


def core_pass(plan: Plan, params: Params, mode: int, lr: float, lam: float):
    check(plan._lib.ft_core_pass(plan.handle, _p(plan, params), int(mode), float(lr), float(lam), _stream()))


def core_epoch(plan: Plan, params: Params, lr: float, lam: float):
    check(plan._lib.ft_core_epoch(plan.handle, _p(plan, params), float(lr), float(lam), _stream()))


def epoch(plan: Plan, params: Params, lr_a: float, lam_a: float, lr_b: float, lam_b: float):
    check(plan._lib.ft_epoch(plan.handle, _p(plan, params), float(lr_a), float(lam_a), float(lr_b), float(lam_b),
                             _stream()))


def loss(plan: Plan, params: Params, lam_a: float = 0.0, lam_b: float = 0.0, out=None):
    """Device float64 tensor [SSE, RMSE, lam_a sum ||A||^2, lam_b sum ||B||^2]."""
    import torch

    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=params.A[0].device)
    _device_vector(out, "out", 4, torch.float64)
    check(plan._lib.ft_loss(plan.handle, _p(plan, params), float(lam_a), float(lam_b), out.data_ptr(), _stream()))
    return out


def loss_noalloc(plan: Plan, params: Params, lam_a: float = 0.0, lam_b: float = 0.0, out=None):
    """As loss(), through ft_loss_noalloc: no scratch from the caller, nothing allocated by the library (the
    partial sums live in its static device array).  `out` (float64 CUDA tensor of 4) is written in place;
    give one to keep this call free of torch allocations too."""
    import torch

    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=params.A[0].device)
    _device_vector(out, "out", 4, torch.float64)
    if plan.workspace is None:
        raise RuntimeError("plan not uploaded")
    s = params.struct(plan, with_scratch=False)
    check(plan._lib.ft_loss_noalloc(plan.handle, ctypes.byref(s), float(lam_a), float(lam_b), out.data_ptr(),
                                    _stream()))
    return out


def forward(plan: Plan, params: Params, out=None):
    """xhat of every element in input order (plan built with with_perm=True)."""
    import torch

    if out is None:
        out = torch.empty(plan.nnz, dtype=torch.float32, device=params.A[0].device)
    _device_vector(out, "out", plan.nnz, torch.float32)
    check(plan._lib.ft_forward(plan.handle, _p(plan, params), out.data_ptr(), _stream()))
    return out


def grad(plan: Plan, params: Params, upstream=None):
    """(dA list, dB list) for dL/dxhat = upstream (input order), or of 1/2 sum e^2 when upstream is None."""
    import torch

    gA = [torch.empty_like(a) for a in params.A]
    gB = [torch.empty_like(b) for b in params.B]
    arrA = (ctypes.c_void_p * len(gA))(*[t.data_ptr() for t in gA])
    arrB = (ctypes.c_void_p * len(gB))(*[t.data_ptr() for t in gB])
    up = None
    if upstream is not None:
        upstream = upstream.contiguous().to(torch.float32)
        _device_vector(upstream, "upstream", plan.nnz, torch.float32)
        up = upstream.data_ptr()
    check(plan._lib.ft_grad(plan.handle, _p(plan, params), up, arrA, arrB, _stream()))
    return gA, gB
