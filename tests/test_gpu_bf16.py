"""BF16 storage (FP32 masters, BF16 copies of A, B, C, FP32 accumulation) against the FP64 oracle.

Error model: every stored BF16 value is within 2^-9 relative of its master, so
|C16 - A B| <= 1.5 2^-8 S with S = |A| |B|, and a prediction (a product of N such factors summed
over r) is within 1.5 N 2^-8 sum_r prod_n S; the tests allow 2 N 2^-8 of that scale.  Updates
take their data term from BF16 quantities (relative error up to about (N + 1) 2^-8) while the
decay acts on the FP32 masters exactly.
"""
import numpy as np
import pytest

from tests.gpu_common import bf16_scale, delta_ok, gpu_setup, make_problem, oracle_model, to_np

pytestmark = pytest.mark.gpu

CASES = [
    ("uniform3_j8", [1000, 1000, 1000], 100_000, 0.0, 8, 8, {}),
    ("zipf3_j16", [3000, 400, 60], 200_000, 1.1, 16, 16, {}),
    ("zipf3_j32", [1500, 200, 40], 60_000, 1.1, 32, 32, {"chunk": 32, "fanin": 8}),
    ("zipf4_j32", [500, 300, 100, 40], 40_000, 1.1, 32, 32, {}),
    ("zipf8_j8r16", [30, 25, 20, 20, 15, 15, 10, 10], 40_000, 1.05, 8, 16, {"chunk": 40}),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def problem(request):
    name, dims, nnz, zipf, J, R, kw = request.param
    vk = "normal3" if len(dims) == 8 else "int1to5"
    c, v, A, B = make_problem(dims, nnz, zipf, J, R, seed=13, values=vk)
    print(f"\n[bf16 case {name}] dims={dims} nnz={nnz} J={J} R={R} plan={kw}", flush=True)
    return name, dims, J, R, c, v, A, B, kw


def test_casts_and_refresh(problem):
    import torch

    name, dims, J, R, c, v, A, B, kw = problem
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, storage="bf16", **kw)
    torch.cuda.synchronize()
    for n in range(len(dims)):
        # the cast kernel rounds to nearest even exactly as torch does
        assert torch.equal(prm.A16[n], prm.A[n].to(torch.bfloat16)), (name, n)
        assert torch.equal(prm.B16[n], prm.B[n].to(torch.bfloat16)), (name, n)
        a16 = prm.A16[n].float().cpu().double().numpy()
        b16 = prm.B16[n].float().cpu().double().numpy()
        exact = a16 @ b16
        got = prm.C16[n].float().cpu().double().numpy()
        # FP32 accumulation then one rounding to BF16: within one BF16 ulp of the exact product
        ulp = np.maximum(np.abs(exact), 1e-38) * 2.0 ** -7
        assert np.all(np.abs(got - exact) <= ulp), (name, n)


def test_predict_and_loss(problem):
    import torch

    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, kw = problem
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, storage="bf16", **kw)
    orc = oracle_model(dims, J, R, c, v, A, B)
    q = np.ascontiguousarray(c[:, :20000])
    got = to_np(ft.predict(plan, prm, torch.from_numpy(q).cuda()))
    want = orc.predict(q)
    N = len(dims)
    assert np.all(np.abs(got - want) <= 2 * N * 2.0 ** -8 * bf16_scale(A, B, q)), name
    out = to_np(ft.loss(plan, prm, 1e-2, 1e-2))
    ref = orc.loss(1e-2, 1e-2)
    # SSE is dominated by (x - xhat) with |xhat| << |x| at this initialisation
    np.testing.assert_allclose(out[0], ref[0], rtol=1e-3)
    np.testing.assert_allclose(out[2:], ref[2:], rtol=1e-6)  # regularisers use the FP32 masters


def test_factor_and_core_passes(problem):
    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, kw = problem
    N = len(dims)
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, storage="bf16", **kw)
    orc = oracle_model(dims, J, R, c, v, A, B)
    tol = 4 * (N + 1) * 2.0 ** -8
    for lam in (1e-2, 0.0):
        plan, prm = gpu_setup(dims, J, R, c, v, A, B, storage="bf16", **kw)
        orc = oracle_model(dims, J, R, c, v, A, B)
        for m in range(N):
            before = orc.A[m].copy()
            ft.factor_pass(plan, prm, m, 1e-3, lam)
            orc.factor_pass(m, 1e-3, lam)
            ok, err, bound = delta_ok(to_np(prm.A[m]), orc.A[m], before, rel=tol)
            assert ok, (name, lam, m, err, bound)
            ft.refresh(plan, prm, m)
            orc.refresh(m)
    for m in range(N):
        before = orc.B[m].copy()
        ft.core_pass(plan, prm, m, 1e-3, 1e-2)
        orc.core_pass(m, 1e-3, 1e-2)
        ok, err, bound = delta_ok(to_np(prm.B[m]), orc.B[m], before, rel=tol)
        assert ok, (name, "core", m, err, bound)
        ft.refresh(plan, prm, m)
        orc.refresh(m)


def test_rmse_matches_fp32_and_repeatable():
    """Learning regime (sigma 0.5, lr 1e-2, uniform coordinates, where the serial method converges; on long
    Zipf rows these steps diverge in FP64 as well): BF16 storage reaches the FP32 RMSE within 0.5 %."""
    import torch

    import paper_2210_06014_amd as ft

    dims, J, R = [1000, 1000, 1000], 8, 8
    c, v, A, B = make_problem(dims, 100_000, 0.0, J, R, seed=21, sigma=0.5)
    plan, p32 = gpu_setup(dims, J, R, c, v, A, B)
    p16 = ft.Params(A, B, storage="bf16")
    ft.refresh(plan, p16)
    twin = p16.clone()
    r0 = float(ft.loss(plan, p32)[1])
    for e in range(3):
        ft.epoch(plan, p32, 1e-2, 1e-2, 1e-2, 1e-2)
        ft.epoch(plan, p16, 1e-2, 1e-2, 1e-2, 1e-2)
        ft.epoch(plan, twin, 1e-2, 1e-2, 1e-2, 1e-2)
    r32 = float(ft.loss(plan, p32)[1])
    r16 = float(ft.loss(plan, p16)[1])
    assert r32 < 0.95 * r0, (r0, r32)
    assert abs(r16 - r32) <= 5e-3 * r32, (r16, r32)
    torch.cuda.synchronize()
    for n in range(3):
        assert torch.equal(twin.A[n], p16.A[n]) and torch.equal(twin.B[n], p16.B[n])
