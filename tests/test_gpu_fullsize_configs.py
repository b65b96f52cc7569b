"""Full-size parity for the other workloads, on outputs the oracle can compute piecewise.

* Netflix-shaped, J = R = 32, FP32 and BF16 storage: one factor pass per mode on sampled rows.
* Order 8, every dim 10000, 50M elements, J = 8, R = 16 (FP32 and BF16): factor passes on sampled rows.
* Order 4, 1e6 x 1e5 x 1e4 x 1e3, 200M elements, J = R = 32, BF16 storage, as an autograd function:
  predictions of sampled elements, and the gradient rows dA(n)[i] of sampled rows (a row of dA depends only
  on the elements of that row, so the oracle runs on exactly those elements).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import bf16_scale, delta_ok, to_np

pytestmark = pytest.mark.gpu


def _sample_rows(counts, plan, m, max_len=None):
    """The longest rows and rows near the piece boundaries of mode m's plan (head, then chunks)."""
    info = plan.mode_info(m)
    head, chunk = info["head"], info["chunk"]
    order = np.argsort(-counts, kind="stable")
    if max_len is not None:
        order = order[counts[order] <= max_len]
    picks = [order[0], order[min(7, len(order) - 1)]]
    for target in (head + chunk * 2 + 3, head + 1, head // 2, chunk + 1, 2):
        picks.append(np.argsort(np.abs(counts - target), kind="stable")[0])
    return np.unique(np.array(picks))


def _factor_sampled(w, c, v, plan, prm, tol):
    import torch

    import paper_2210_06014_amd as ft

    N = len(w.dims)
    for m in range(N):
        A_now = [to_np(a) for a in prm.A]
        B_now = [to_np(b) for b in prm.B]
        ft.factor_pass(plan, prm, m, w.lr, w.lam)
        torch.cuda.synchronize()
        counts = np.bincount(c[m], minlength=w.dims[m])
        rows = _sample_rows(counts, plan, m)
        sel = np.isin(c[m], rows)
        print(f"[fullsize {w.name}] mode {m}: lengths {counts[rows].tolist()}", flush=True)
        orc = oracle.Model(w.dims, w.J, w.R, np.ascontiguousarray(c[:, sel]), v[sel].astype(np.float64), A_now, B_now)
        orc.factor_pass(m, w.lr, w.lam)
        got = to_np(prm.A[m])[rows]
        for k, i in enumerate(rows):
            ok, err, bound = delta_ok(got[k], orc.A[m][i], A_now[m][i], rel=tol)
            assert ok, (w.name, m, int(i), int(counts[i]), err, bound)
        ft.refresh(plan, prm, m)


@pytest.mark.parametrize("workload", ["netflix32", "order8"])
def test_factor_pass_fullsize(workload):
    import paper_2210_06014_amd as ft

    w = synth.WORKLOADS[workload]
    print(f"\n[fullsize] generating {workload}", flush=True)
    c, v, A, B = synth.make(w)
    plan = ft.Plan(w.dims, w.J[0], w.R, c, v)
    for storage, tol in (("f32", 1e-3), ("bf16", 4 * (len(w.dims) + 1) * 2.0 ** -8)):
        prm = ft.Params(A, B, storage=storage)
        ft.refresh(plan, prm)
        _factor_sampled(w, c, v, plan, prm, tol)
        del prm
    plan.close()


def test_order4_autograd_fullsize():
    import torch

    import paper_2210_06014_amd as ft

    w = synth.WORKLOADS["order4"]
    print("\n[fullsize] generating order4 200M", flush=True)
    c, v, A, B = synth.make(w)
    N = len(w.dims)
    plan = ft.Plan(w.dims, w.J[0], w.R, c, v, with_perm=True)
    At = [torch.tensor(a, device="cuda", requires_grad=True) for a in A]
    Bt = [torch.tensor(b, device="cuda", requires_grad=True) for b in B]
    xhat = ft.reconstruct(plan, At, Bt, storage="bf16")
    x = torch.from_numpy(v).cuda()
    loss = 0.5 * torch.sum((xhat - x) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    pick = rng.choice(c.shape[1], size=20000, replace=False)
    q = np.ascontiguousarray(c[:, pick])
    A64 = [a.astype(np.float64) for a in A]
    B64 = [b.astype(np.float64) for b in B]
    orc = oracle.Model(w.dims, w.J, w.R, q, v[pick].astype(np.float64), A64, B64)
    want = orc.predict(q)
    got = to_np(xhat)[pick]
    assert np.all(np.abs(got - want) <= 2 * N * 2.0 ** -8 * bf16_scale(A, B, q))
    # gradient rows: dA(n)[i] = sum_{x in row i} -(x - xhat_x) g(n)_x
    for n in range(N):
        counts = np.bincount(c[n], minlength=w.dims[n])
        rows = _sample_rows(counts, plan, n, max_len=100_000)
        sel = np.isin(c[n], rows)
        print(f"[fullsize order4] mode {n}: gradient rows with lengths {counts[rows].tolist()}", flush=True)
        sub = oracle.Model(w.dims, w.J, w.R, np.ascontiguousarray(c[:, sel]), v[sel].astype(np.float64), A64, B64)
        rA, _ = sub.grad()
        g = to_np(At[n].grad)[rows]
        r = rA[n][rows]
        # BF16 inputs: per-element error of delta and g of order (N + 1) 2^-8, summed over the row
        for k in range(len(rows)):
            scale = np.linalg.norm(r[k]) + 1e-30
            assert np.linalg.norm(g[k] - r[k]) <= 8 * (N + 1) * 2.0 ** -8 * scale + 1e-6, (n, int(rows[k]))
    plan.close()
