"""ft_loss_noalloc: the loss with its partial sums in the library's static device array, no caller scratch.

Called through the C-ABI (the binding only marshals) and compared with ft_loss on the same plan and
parameters: same kernels and launch grid, so the four FP64 results must be identical.  Two calls in a row,
the second on a smaller plan (fewer segments, so fewer loss partials): the array keeps the first call's
contents, which the second must not pick up.  Also with BF16 storage, and with the scratch pointer NULL.
"""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import gpu_setup, make_problem

pytestmark = pytest.mark.gpu

CASES = [([3000, 400, 60], 200_000, 16, 16, 21), ([500, 300, 40], 20_000, 8, 8, 22)]


def _both(ft, plan, prm, lam):
    import torch

    from paper_2210_06014_amd import _lib

    ref = ft.loss(plan, prm, lam, lam)
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    s = prm.struct(plan, with_scratch=False)
    assert s.scratch is None and s.scratch_bytes == 0
    st = plan._lib.ft_loss_noalloc(plan.handle, ctypes.byref(s), lam, lam, out.data_ptr(),
                                   torch.cuda.current_stream().cuda_stream)
    _lib.check(st)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_noalloc_loss_matches_loss(storage):
    import paper_2210_06014_amd as ft

    for dims, nnz, J, R, seed in CASES:
        print(f"[no-alloc] storage={storage} dims={dims} nnz={nnz} J={J} R={R} seed={seed}", flush=True)
        c, v, A, B = make_problem(dims, nnz, 1.1, J, R, seed=seed)
        plan, prm = gpu_setup(dims, J, R, c, v, A, B, storage=storage)
        ft.epoch(plan, prm, 1e-3, 1e-2, 1e-3, 1e-2)
        ref, got = _both(ft, plan, prm, 1e-2)
        assert np.all(np.isfinite(ref)) and ref[0] > 0
        np.testing.assert_array_equal(got, ref)
        # the binding's wrapper gives the same
        np.testing.assert_array_equal(ft.loss_noalloc(plan, prm, 1e-2, 1e-2).cpu().numpy(), ref)


def test_noalloc_loss_refuses_bad_arguments():
    import torch

    import paper_2210_06014_amd as ft
    from paper_2210_06014_amd import _lib

    dims, nnz, J, R, seed = CASES[1]
    c, v, A, B = make_problem(dims, nnz, 1.1, J, R, seed=seed)
    plan, prm = gpu_setup(dims, J, R, c, v, A, B)
    s = prm.struct(plan, with_scratch=False)
    st = plan._lib.ft_loss_noalloc(plan.handle, ctypes.byref(s), 0.0, 0.0, None,
                                   torch.cuda.current_stream().cuda_stream)
    assert _lib.STATUS[st] == "FT_ERR_ARG"
    with pytest.raises(ValueError):
        ft.loss_noalloc(plan, prm, out=torch.empty(3, dtype=torch.float64, device="cuda"))
