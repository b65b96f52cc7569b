"""GPU (HIP, FP32) against the FP64 oracle on the same seeded inputs, through the C-ABI.

Tolerances (FP32 kernels against FP64, derivation in the design notes):
  predictions     |d xhat| <= 1e-5 * sum_r prod_n |C(n)[i_n, r]|  and  ||d xhat|| <= 1e-5 ||xhat||
  C refresh       |d C|    <= 1e-5 * sum_j |A[i, j] B[j, r]|
  gradients       ||d G|| <= 1e-4 ||G||  per mode
  one pass        ||P_gpu - P_orc|| <= 1e-3 ||P_orc - P_before|| + 1e-6 ||P_orc||
  loss, RMSE      relative 1e-5 (SSE), final RMSE after epochs within 0.5 %
"""
import numpy as np
import pytest

from tests.gpu_common import abs_scale, delta_ok, gpu_setup, make_problem, oracle_model, to_np

pytestmark = pytest.mark.gpu

# (name, dims, nnz, zipf, J, R, plan kwargs)
CASES = [
    ("uniform3_j8", [1000, 1000, 1000], 100_000, 0.0, 8, 8, {}),
    ("zipf3_j16", [3000, 400, 60], 200_000, 1.1, 16, 16, {}),
    ("zipf3_j16_smallchunk", [3000, 400, 60], 60_000, 1.1, 16, 16, {"chunk": 16, "fanin": 4}),
    ("zipf3_j32", [1500, 200, 40], 60_000, 1.1, 32, 32, {"chunk": 32, "fanin": 8}),
    ("zipf4_j8", [400, 300, 200, 50], 80_000, 1.1, 8, 8, {"chunk": 24, "fanin": 3}),
    ("zipf4_j32", [500, 300, 100, 40], 40_000, 1.1, 32, 32, {"chunk": 64, "head": 256}),
    ("zipf8_j8r16", [30, 25, 20, 20, 15, 15, 10, 10], 40_000, 1.05, 8, 16, {"chunk": 40}),
]
IDS = [c[0] for c in CASES]


@pytest.fixture(scope="module", params=CASES, ids=IDS)
def problem(request):
    name, dims, nnz, zipf, J, R, kw = request.param
    vk = "normal3" if len(dims) == 8 else "int1to5"
    c, v, A, B = make_problem(dims, nnz, zipf, J, R, seed=11, values=vk)
    print(f"\n[case {name}] dims={dims} nnz={nnz} J={J} R={R} plan={kw}", flush=True)
    return name, dims, J, R, c, v, A, B, kw


def test_refresh(problem):
    name, dims, J, R, c, v, A, B, kw = problem
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, **kw)
    for n in range(len(dims)):
        want = A[n].astype(np.float64) @ B[n].astype(np.float64)
        scale = np.abs(A[n].astype(np.float64)) @ np.abs(B[n].astype(np.float64))
        got = to_np(prm.C[n])
        assert np.all(np.abs(got - want) <= 1e-5 * scale + 1e-30), name


def test_predict_and_loss(problem):
    import torch

    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, kw = problem
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, **kw)
    orc = oracle_model(dims, J, R, c, v, A, B)
    # queries: the stored elements plus random coordinates (not necessarily stored)
    rng = np.random.default_rng(3)
    rnd = np.stack([rng.integers(0, d, size=5000) for d in dims]).astype(np.int32)
    q = np.concatenate([c[:, :20000], rnd], axis=1)
    got = to_np(ft.predict(plan, prm, torch.from_numpy(q).cuda()))
    want = orc.predict(q)
    scale = abs_scale(orc.C, q)
    assert np.all(np.abs(got - want) <= 1e-5 * scale + 1e-30), name
    assert np.linalg.norm(got - want) <= 1e-5 * np.linalg.norm(want)
    out = to_np(ft.loss(plan, prm, 1e-2, 2e-2))
    ref = orc.loss(1e-2, 2e-2)
    np.testing.assert_allclose(out, ref, rtol=1e-5)


def test_core_gradient(problem):
    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, kw = problem
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, **kw)
    orc = oracle_model(dims, J, R, c, v, A, B)
    for m in range(len(dims)):
        G = to_np(ft.core_grad(plan, prm, m))
        Gr = orc.core_grad(m)
        assert np.linalg.norm(G - Gr) <= 1e-4 * np.linalg.norm(Gr), (name, m)


@pytest.mark.parametrize("lam", [1e-2, 0.0])
def test_factor_pass_each_mode(problem, lam):
    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, kw = problem
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, **kw)
    orc = oracle_model(dims, J, R, c, v, A, B)
    lr = 1e-3
    for m in range(len(dims)):
        before = orc.A[m].copy()
        ft.factor_pass(plan, prm, m, lr, lam)
        orc.factor_pass(m, lr, lam)
        ok, err, bound = delta_ok(to_np(prm.A[m]), orc.A[m], before)
        assert ok, (name, m, err, bound)
        # keep both sides on the same state for the next mode
        ft.refresh(plan, prm, m)
        orc.refresh(m)


def test_core_pass_each_mode(problem):
    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, kw = problem
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, **kw)
    orc = oracle_model(dims, J, R, c, v, A, B)
    for m in range(len(dims)):
        before = orc.B[m].copy()
        ft.core_pass(plan, prm, m, 1e-3, 1e-2)
        orc.core_pass(m, 1e-3, 1e-2)
        ok, err, bound = delta_ok(to_np(prm.B[m]), orc.B[m], before)
        assert ok, (name, m, err, bound)
        ft.refresh(plan, prm, m)
        orc.refresh(m)


def test_gradients(problem):
    import torch

    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, kw = problem
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, with_perm=True, **kw)
    orc = oracle_model(dims, J, R, c, v, A, B)
    gA, gB = ft.grad(plan, prm)
    rA, rB = orc.grad()
    for n in range(len(dims)):
        assert np.linalg.norm(to_np(gA[n]) - rA[n]) <= 1e-4 * np.linalg.norm(rA[n]), (name, "A", n)
        assert np.linalg.norm(to_np(gB[n]) - rB[n]) <= 1e-4 * np.linalg.norm(rB[n]), (name, "B", n)
    delta = np.random.default_rng(5).normal(size=c.shape[1]).astype(np.float32)
    gA, gB = ft.grad(plan, prm, torch.from_numpy(delta).cuda())
    rA, rB = orc.grad(delta.astype(np.float64))
    for n in range(len(dims)):
        assert np.linalg.norm(to_np(gA[n]) - rA[n]) <= 1e-4 * np.linalg.norm(rA[n]), (name, "A*", n)
        assert np.linalg.norm(to_np(gB[n]) - rB[n]) <= 1e-4 * np.linalg.norm(rB[n]), (name, "B*", n)
    xh = to_np(ft.forward(plan, prm))
    want = orc.predict(c)
    assert np.all(np.abs(xh - want) <= 1e-5 * abs_scale(orc.C, c) + 1e-30)


def test_epochs_and_determinism(problem):
    import torch

    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, kw = problem
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, **kw)
    orc = oracle_model(dims, J, R, c, v, A, B)
    A0 = [a.astype(np.float64) for a in A]
    B0 = [b.astype(np.float64) for b in B]
    twin = prm.clone()
    for e in range(2):
        ft.epoch(plan, prm, 1e-3, 1e-2, 1e-3, 1e-2)
        orc.epoch(1e-3, 1e-2, 1e-3, 1e-2)
    for n in range(len(dims)):
        ok, err, bound = delta_ok(to_np(prm.A[n]), orc.A[n], A0[n])
        assert ok, (name, "A", n, err, bound)
        ok, err, bound = delta_ok(to_np(prm.B[n]), orc.B[n], B0[n])
        assert ok, (name, "B", n, err, bound)
    rm = to_np(ft.loss(plan, prm))[1]
    assert abs(rm - orc.loss()[1]) <= 5e-3 * orc.loss()[1]
    # bitwise repeatability
    for e in range(2):
        ft.epoch(plan, twin, 1e-3, 1e-2, 1e-3, 1e-2)
    torch.cuda.synchronize()
    for n in range(len(dims)):
        assert torch.equal(twin.A[n], prm.A[n]) and torch.equal(twin.B[n], prm.B[n]), (name, n)


def test_learning_regime_rmse():
    """Larger steps (sigma 0.5, lr 1e-2) where the RMSE really moves: GPU and oracle agree on the curve."""
    import paper_2210_06014_amd as ft

    dims, J, R = [1000, 1000, 1000], 8, 8
    c, v, A, B = make_problem(dims, 100_000, 0.0, J, R, seed=21, sigma=0.5)
    plan, prm = gpu_setup(dims, J, R, c, v, A, B)
    orc = oracle_model(dims, J, R, c, v, A, B)
    r0 = orc.loss()[1]
    for e in range(3):
        ft.epoch(plan, prm, 1e-2, 1e-2, 1e-2, 1e-2)
        orc.epoch(1e-2, 1e-2, 1e-2, 1e-2)
        g, o = to_np(ft.loss(plan, prm))[1], orc.loss()[1]
        assert abs(g - o) <= 5e-3 * o, (e, g, o)
    assert orc.loss()[1] < 0.95 * r0


def test_empty_and_tiny():
    import paper_2210_06014_amd as ft

    dims, J, R = [7, 5, 3], 8, 8
    c = np.zeros((3, 0), dtype=np.int32)
    v = np.zeros(0, dtype=np.float32)
    _, _, A, B = make_problem(dims, 10, 0.0, J, R, seed=2)
    plan, prm = gpu_setup(dims, J, R, c, v, A, B)
    ft.epoch(plan, prm, 1e-3, 1e-2, 1e-3, 1e-2)
    for n in range(3):
        np.testing.assert_array_equal(to_np(prm.A[n]), A[n])
        np.testing.assert_array_equal(to_np(prm.B[n]), B[n])
    out = to_np(ft.loss(plan, prm))
    assert out[0] == 0 and out[1] == 0
    # a single element
    c1 = np.array([[6], [4], [2]], dtype=np.int32)
    v1 = np.array([3.0], dtype=np.float32)
    plan, prm = gpu_setup(dims, J, R, c1, v1, A, B)
    orc = oracle_model(dims, J, R, c1, v1, A, B)
    ft.epoch(plan, prm, 0.1, 0.1, 0.1, 0.1)
    orc.epoch(0.1, 0.1, 0.1, 0.1)
    for n in range(3):
        np.testing.assert_allclose(to_np(prm.A[n]), orc.A[n], rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(to_np(prm.B[n]), orc.B[n], rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("case", ["zipf3_j16", "zipf3_j32", "zipf4_j8"])
def test_fiber_shared_g_is_bitwise_equal(case):
    """Sharing g per fiber (Section 3.2) changes where g is computed, not how: results are bit-identical."""
    import torch

    import paper_2210_06014_amd as ft

    name, dims, nnz, zipf, J, R, kw = [c for c in CASES if c[0] == case][0]
    dims = [max(d // 4, 2) for d in dims]  # denser: longer fibers
    c, v, A, B = make_problem(dims, nnz, zipf, J, R, seed=17)
    outs = []
    for share in (True, False):
        for storage in ("f32", "bf16"):
            plan, prm = gpu_setup(dims, J, R, c, v, A, B, storage=storage, fiber_share=share, **kw)
            if share:
                assert any(plan.mode_info(m)["fiber_shared"] for m in range(len(dims)))
            ft.epoch(plan, prm, 1e-3, 1e-2, 1e-3, 1e-2)
            torch.cuda.synchronize()
            outs.append([t.clone() for t in prm.A + prm.B])
    for a, b in zip(outs[0], outs[2]):
        assert torch.equal(a, b)
    for a, b in zip(outs[1], outs[3]):
        assert torch.equal(a, b)


@pytest.mark.parametrize("case", ["zipf3_j16_smallchunk", "zipf3_j32", "zipf4_j8", "zipf8_j8r16"])
def test_fused_factor_launch_is_bitwise_equal(case):
    """The exact factor pass launches its in-place items and its chunk maps as one kernel by default; as two
    kernels in sequence (FT_SPLIT_FACTOR) every item runs the same code, so the results are bit-identical.
    Also with long heads (rows of up to 4 chunks in place), which move elements from the maps to the chains."""
    import torch

    import paper_2210_06014_amd as ft

    name, dims, nnz, zipf, J, R, kw = [c for c in CASES if c[0] == case][0]
    vk = "normal3" if len(dims) == 8 else "int1to5"
    c, v, A, B = make_problem(dims, nnz, zipf, J, R, seed=19, values=vk)
    chunk = kw.get("chunk", 512)
    for head in (0, 4 * chunk):
        outs = []
        for fused in (True, False):
            for storage in ("f32", "bf16"):
                plan, prm = gpu_setup(dims, J, R, c, v, A, B, storage=storage, fused=fused, **kw,
                                      **({"head": head} if head else {}))
                assert sum(plan.mode_info(m)["heavy_rows"] for m in range(len(dims))) > 0
                ft.epoch(plan, prm, 1e-3, 1e-2, 1e-3, 1e-2)
                torch.cuda.synchronize()
                outs.append([t.clone() for t in prm.A + prm.B])
        for a, b in zip(outs[0], outs[2]):
            assert torch.equal(a, b), (name, head, "f32")
        for a, b in zip(outs[1], outs[3]):
            assert torch.equal(a, b), (name, head, "bf16")


@pytest.mark.parametrize("case", ["zipf3_j16", "zipf3_j16_smallchunk"])
def test_no_c_cache_variant(case):
    """FT_NO_C_CACHE (the FastTucker cost, Table 5): every C row formed from A and B on use; same results."""
    import paper_2210_06014_amd as ft

    name, dims, nnz, zipf, J, R, kw = [c for c in CASES if c[0] == case][0]
    c, v, A, B = make_problem(dims, nnz, zipf, J, R, seed=11)
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, c_cache=False, **kw)
    orc = oracle_model(dims, J, R, c, v, A, B)
    for m in range(3):
        before = orc.A[m].copy()
        ft.factor_pass(plan, prm, m, 1e-3, 1e-2)
        orc.factor_pass(m, 1e-3, 1e-2)
        ok, err, bound = delta_ok(to_np(prm.A[m]), orc.A[m], before)
        assert ok, (name, "factor", m, err, bound)
        ft.refresh(plan, prm, m)
        orc.refresh(m)
    for m in range(3):
        before = orc.B[m].copy()
        ft.core_pass(plan, prm, m, 1e-3, 1e-2)
        orc.core_pass(m, 1e-3, 1e-2)
        ok, err, bound = delta_ok(to_np(prm.B[m]), orc.B[m], before)
        assert ok, (name, "core", m, err, bound)
        ft.refresh(plan, prm, m)
        orc.refresh(m)


@pytest.mark.parametrize("head", [1, 7, 1 << 30])
def test_factor_pass_head_lengths(head):
    """Rows split after `head` serial elements (1: every row of two or more elements is heavy; 2^30: none is)."""
    import paper_2210_06014_amd as ft

    dims, J, R = [300, 40, 12], 16, 16
    c, v, A, B = make_problem(dims, 30_000, 1.1, J, R, seed=23)
    plan, prm = gpu_setup(dims, J, R, c, v, A, B, chunk=16, head=head, fanin=3)
    heavy = [plan.mode_info(m)["heavy_rows"] for m in range(3)]
    assert (sum(heavy) == 0) == (head == 1 << 30)
    orc = oracle_model(dims, J, R, c, v, A, B)
    for m in range(3):
        before = orc.A[m].copy()
        ft.factor_pass(plan, prm, m, 1e-3, 1e-2)
        orc.factor_pass(m, 1e-3, 1e-2)
        ok, err, bound = delta_ok(to_np(prm.A[m]), orc.A[m], before)
        assert ok, (head, m, err, bound)
        ft.refresh(plan, prm, m)
        orc.refresh(m)
