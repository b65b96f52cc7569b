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


def test_autograd_bf16_finite_difference_order4_slice():
    """The differentiable form at the order-4 workload's shape (1e6 x 1e5 x 1e4 x 1e3, J = R = 32, BF16 storage):
    the first 10k elements its generator draws (coordinates are the first distinct draws in draw order, values
    a counter-based stream, so these are the first 10k elements of the full tensor), loss 1/2 sum e^2.  The
    directional derivative of autograd is checked against FP64 central differences of the oracle's loss.

    Tolerance from the BF16 error model: A16, B16 are within 2^-9 of the masters and C16 = bf16(A16 B16) within
    1.5 2^-8 of A B (products of positive factors); a term of the derivative, delta_x times a product of N - 1
    C16 rows and one B16 (or A16) entry, is then within (1.5 (N - 1) + 0.5) 2^-8 of its exact value, and delta_x
    = xhat_x - x_x is dominated by x_x.  Parameters and direction are positive (absolute values of the seeded
    draws), so every term has the same sign and the sum keeps the terms' relative bound: |ad - fd| <=
    1.5 N 2^-8 |fd|.  With signed parameters the terms cancel and the same model bounds nothing useful."""
    import torch

    import oracle
    import paper_2210_06014_amd as ft
    import synth

    w = synth.WORKLOADS["order4"]
    dims, J, R, N = w.dims, w.J[0], w.R, len(w.dims)
    c, _ = synth.coords(dims, 10_000, w.zipf, w.seed)
    v = synth.values(10_000, w.value_kind, w.seed)
    A, B = synth.init_params(dims, J, R, w.sigma, w.seed + 1)
    A = [np.abs(a) for a in A]
    B = [np.abs(b) for b in B]
    plan = ft.Plan(dims, J, R, c, v, with_perm=True)
    At = [torch.tensor(a, device="cuda", requires_grad=True) for a in A]
    Bt = [torch.tensor(b, device="cuda", requires_grad=True) for b in B]
    x = torch.tensor(v, device="cuda")
    loss = 0.5 * torch.sum((ft.reconstruct(plan, At, Bt, storage="bf16") - x) ** 2)
    loss.backward()
    rng = np.random.default_rng(5)
    dA = [np.abs(rng.normal(size=a.shape)) for a in A]
    dB = [np.abs(rng.normal(size=b.shape)) for b in B]
    ad = sum(float(np.sum(to_np(t.grad) * d)) for t, d in zip(At, dA)) + sum(
        float(np.sum(to_np(t.grad) * d)) for t, d in zip(Bt, dB))

    def f(h):
        Ah = [a.astype(np.float64) + h * d for a, d in zip(A, dA)]
        Bh = [b.astype(np.float64) + h * d for b, d in zip(B, dB)]
        m = oracle.Model(dims, J, R, c, v.astype(np.float64), Ah, Bh)
        e = v.astype(np.float64) - m.predict(c)
        return 0.5 * float(np.sum(e * e))

    h = 1e-5
    fd = (f(h) - f(-h)) / (2 * h)
    print(f"\n[bf16 fd] autograd {ad:.8e} central difference {fd:.8e} rel {abs(ad - fd) / abs(fd):.3e}", flush=True)
    assert abs(ad - fd) <= 1.5 * N * 2.0 ** -8 * abs(fd), (ad, fd)
