"""x̂ as a torch.autograd.Function: gradients against the FP64 oracle (itself pinned by finite differences)."""
import numpy as np
import pytest

from tests.gpu_common import abs_scale, make_problem, oracle_model, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,J,R,nnz", [([300, 200, 100, 50], 32, 32, 20_000), ([500, 400, 90], 16, 16, 30_000)])
def test_autograd_matches_oracle(dims, J, R, nnz):
    import torch

    import paper_2210_06014_amd as ft

    c, v, A, B = make_problem(dims, nnz, 1.1, J, R, seed=31)
    plan = ft.Plan(dims, J, R, c, v, with_perm=True)
    At = [torch.tensor(a, device="cuda", requires_grad=True) for a in A]
    Bt = [torch.tensor(b, device="cuda", requires_grad=True) for b in B]
    xhat = ft.reconstruct(plan, At, Bt)
    orc = oracle_model(dims, J, R, c, v, A, B)
    want = orc.predict(c)
    assert np.all(np.abs(to_np(xhat) - want) <= 1e-5 * abs_scale(orc.C, c) + 1e-30)
    # mean squared error: dL/dxhat = 2 (xhat - x) / nnz
    x = torch.tensor(v, device="cuda")
    loss = torch.mean((xhat - x) ** 2)
    loss.backward()
    delta = 2.0 * (want - v.astype(np.float64)) / nnz
    rA, rB = orc.grad(delta)
    for n in range(len(dims)):
        assert np.linalg.norm(to_np(At[n].grad) - rA[n]) <= 1e-4 * np.linalg.norm(rA[n]), ("A", n)
        assert np.linalg.norm(to_np(Bt[n].grad) - rB[n]) <= 1e-4 * np.linalg.norm(rB[n]), ("B", n)


def test_autograd_finite_difference_slice():
    """Directional derivative of the loss along a random direction: autograd vs central differences in FP64
    computed by the oracle's predictions (10k-element slice of an order-4 Zipf tensor)."""
    import torch

    import oracle
    import paper_2210_06014_amd as ft

    dims, J, R = [1000, 500, 200, 50], 32, 32
    c, v, A, B = make_problem(dims, 10_000, 1.1, J, R, seed=41)
    plan = ft.Plan(dims, J, R, c, v, with_perm=True)
    At = [torch.tensor(a, device="cuda", requires_grad=True) for a in A]
    Bt = [torch.tensor(b, device="cuda", requires_grad=True) for b in B]
    x = torch.tensor(v, device="cuda")
    loss = 0.5 * torch.sum((ft.reconstruct(plan, At, Bt) - x) ** 2)
    loss.backward()
    rng = np.random.default_rng(0)
    dA = [rng.normal(size=a.shape) for a in A]
    dB = [rng.normal(size=b.shape) for b in B]
    ad = sum(float(np.sum(to_np(t.grad) * d)) for t, d in zip(At, dA)) + sum(
        float(np.sum(to_np(t.grad) * d)) for t, d in zip(Bt, dB))

    def f(h):
        Ah = [a.astype(np.float64) + h * d for a, d in zip(A, dA)]
        Bh = [b.astype(np.float64) + h * d for b, d in zip(B, dB)]
        m = oracle.Model(dims, J, R, c, v.astype(np.float64), Ah, Bh)
        e = v.astype(np.float64) - m.predict(c)
        return 0.5 * float(np.sum(e * e))

    h = 1e-4
    fd = (f(h) - f(-h)) / (2 * h)
    assert abs(ad - fd) <= 1e-4 * abs(fd), (ad, fd)
