"""FT_RELAXED factor passes (the chunks of a long row start from the row as its head left it and
are merged under a step guard) against the oracle's relaxed module, element by element.

The tolerance is the one of the exact factor pass: the change of every factor matrix matches the
oracle's to 1e-3 of its size in FP32 storage, 4 (N + 1) 2^-8 in BF16 storage.  One case draws
A, B with sigma 0.35 so that lr sum ||g||^2 exceeds 1 on the long rows and the guard scales
their merged increments.
"""
import numpy as np
import pytest

from tests.gpu_common import delta_ok, gpu_setup, make_problem, oracle_model, to_np

pytestmark = pytest.mark.gpu

CASES = [
    # name, dims, nnz, zipf, J, R, plan, storage, sigma
    ("zipf3_j16", [300, 40, 12], 30_000, 1.1, 16, 16, {"chunk": 16, "head": 40}, "f32", 0.1),
    ("zipf3_j8", [2000, 300, 50], 50_000, 1.1, 8, 8, {"chunk": 32, "head": 64}, "f32", 0.1),
    ("zipf3_j32", [1500, 200, 40], 60_000, 1.1, 32, 32, {"chunk": 32}, "f32", 0.1),
    ("zipf8_j8r16", [30, 25, 20, 20, 15, 15, 10, 10], 40_000, 1.05, 8, 16, {"chunk": 40}, "f32", 0.1),
    ("zipf3_j16_guard", [50, 40, 30], 40_000, 1.1, 16, 16, {"chunk": 64, "head": 128}, "f32", 0.35),
    ("zipf3_j16_bf16", [300, 40, 12], 30_000, 1.1, 16, 16, {"chunk": 16, "head": 40}, "bf16", 0.1),
]

LR, LAM = 1e-3, 1e-2


def _heads(plan):
    info = plan.mode_info(0)
    return info["head"], info["chunk"]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_relaxed_factor_passes(case):
    import paper_2210_06014_amd as ft

    name, dims, nnz, zipf, J, R, kw, storage, sigma = case
    N = len(dims)
    print(f"\n[relaxed case {name}] dims={dims} nnz={nnz} J={J} R={R} plan={kw} {storage}", flush=True)
    c, v, A, B = make_problem(dims, nnz, zipf, J, R, seed=31, sigma=sigma)
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, storage=storage, relaxed=True, **kw)
    assert sum(plan.mode_info(m)["heavy_rows"] for m in range(N)) > 0
    orc = oracle_model(dims, J, R, c, v, A, B)
    head, chunk = _heads(plan)
    if name.endswith("guard"):
        # the longest mode-0 row: lr sum ||g||^2 over its chunked elements is above 1
        w = np.prod([orc.C[n][c[n]] for n in range(1, N)], axis=0)
        gn = np.sum((w @ orc.B[0].T) ** 2, axis=1)
        row = np.argmax(np.bincount(c[0]))
        sel = gn[c[0] == row]
        assert LR * sel.sum() * (sel.size - head) / sel.size > 1.2
    tol = 1e-3 if storage == "f32" else 4 * (N + 1) * 2.0 ** -8
    for m in range(N):
        before = orc.A[m].copy()
        ft.factor_pass(plan, prm, m, LR, LAM)
        orc.factor_pass_relaxed(m, LR, LAM, head, chunk)
        ok, err, bound = delta_ok(to_np(prm.A[m]), orc.A[m], before, rel=tol)
        assert ok, (name, m, err, bound)
        ft.refresh(plan, prm, m)
        orc.refresh(m)


def test_relaxed_epoch_and_loss():
    """One iteration of Algorithm 2 with relaxed factor passes, then the loss."""
    import paper_2210_06014_amd as ft

    dims, J, R, kw = [400, 60, 20], 16, 16, {"chunk": 32, "head": 64}
    c, v, A, B = make_problem(dims, 40_000, 1.1, J, R, seed=32)
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, relaxed=True, **kw)
    orc = oracle_model(dims, J, R, c, v, A, B)
    A0 = [a.copy() for a in orc.A]
    B0 = [b.copy() for b in orc.B]
    ft.epoch(plan, prm, LR, LAM, LR, LAM)
    orc.epoch_relaxed(LR, LAM, LR, LAM, 64, 32)
    for n in range(3):
        ok, err, bound = delta_ok(to_np(prm.A[n]), orc.A[n], A0[n])
        assert ok, ("A", n, err, bound)
        ok, err, bound = delta_ok(to_np(prm.B[n]), orc.B[n], B0[n])
        assert ok, ("B", n, err, bound)
    np.testing.assert_allclose(to_np(ft.loss(plan, prm, LAM, LAM)), orc.loss(LAM, LAM), rtol=1e-4)


def test_relaxed_without_long_rows_is_the_exact_pass():
    """With every row at most `head` long the relaxed plan runs the exact kernels only: same bits."""
    import torch

    import paper_2210_06014_amd as ft

    dims, J, R = [300, 40, 12], 16, 16
    c, v, A, B = make_problem(dims, 30_000, 1.1, J, R, seed=33)
    out = []
    for relaxed in (False, True):
        plan, prm = gpu_setup(dims, J, R, c, v, A, B, relaxed=relaxed, chunk=16, head=1 << 30)
        for m in range(3):
            ft.factor_pass(plan, prm, m, LR, LAM)
            ft.refresh(plan, prm, m)
        torch.cuda.synchronize()
        out.append([prm.A[m].clone() for m in range(3)])
    for m in range(3):
        assert torch.equal(out[0][m], out[1][m]), m


def test_relaxed_is_repeatable():
    """No atomics: two runs from the same parameters give the same bits."""
    import torch

    import paper_2210_06014_amd as ft

    dims, J, R = [300, 40, 12], 16, 16
    c, v, A, B = make_problem(dims, 30_000, 1.1, J, R, seed=34)
    out = []
    for _ in range(2):
        plan, prm = gpu_setup(dims, J, R, c, v, A, B, relaxed=True, chunk=16, head=40)
        for m in range(3):
            ft.factor_pass(plan, prm, m, LR, LAM)
            ft.refresh(plan, prm, m)
        torch.cuda.synchronize()
        out.append([prm.A[m].clone() for m in range(3)])
    for m in range(3):
        assert torch.equal(out[0][m], out[1][m]), m
