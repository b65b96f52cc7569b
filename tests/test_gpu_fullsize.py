"""Parity at the benchmark's full size and launch configuration, on outputs the oracle can compute piecewise.

The Netflix-shaped workload (480000 x 18000 x 2200, 100M elements, Zipf 1.1, J = R = 16) with the
bench's default plan.  Rows are independent within a factor pass, so a sample of rows (the longest row,
rows around the chunk boundary and short rows) is checked against the oracle run on exactly the
elements of those rows, from the same starting state.  The loss is a plain sum the oracle computes over
all 100M elements.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import delta_ok, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def netflix():
    import paper_2210_06014_amd as ft

    w = synth.WORKLOADS["netflix"]
    print("\n[fullsize] generating netflix 100M", flush=True)
    c, v, A, B = synth.make(w)
    plan = ft.Plan(w.dims, w.J[0], w.R, c, v)
    prm = ft.Params(A, B)
    ft.refresh(plan, prm)
    return w, c, v, A, B, plan, prm


def _sample_rows(counts, plan, m):
    """The longest rows and rows near the piece boundaries of mode m's plan (head, then chunks)."""
    info = plan.mode_info(m)
    head, chunk = info["head"], info["chunk"]
    order = np.argsort(-counts, kind="stable")
    picks = [order[0], order[min(5, len(order) - 1)]]
    for target in (head + chunk * 3 + 7, head + 1, head, head // 2, chunk + 1, 3):
        near = np.argsort(np.abs(counts - target), kind="stable")
        picks.append(near[0])
    return np.unique(np.array(picks))


def test_loss_full(netflix):
    import paper_2210_06014_amd as ft

    w, c, v, A, B, plan, prm = netflix
    got = to_np(ft.loss(plan, prm, w.lam, w.lam))
    orc = oracle.Model(w.dims, w.J, w.R, c, v.astype(np.float64), [a.astype(np.float64) for a in A],
                       [b.astype(np.float64) for b in B])
    ref = orc.loss(w.lam, w.lam)
    np.testing.assert_allclose(got, ref, rtol=1e-5)


def test_factor_passes_sampled_rows(netflix):
    import torch

    import paper_2210_06014_amd as ft

    w, c, v, A, B, plan, prm = netflix
    J, R = w.J[0], w.R
    for m in range(3):
        A_now = [to_np(a) for a in prm.A]
        B_now = [to_np(b) for b in prm.B]
        ft.factor_pass(plan, prm, m, w.lr, w.lam)
        torch.cuda.synchronize()
        counts = np.bincount(c[m], minlength=w.dims[m])
        rows = _sample_rows(counts, plan, m)
        sel = np.isin(c[m], rows)
        print(f"[fullsize] mode {m}: rows {rows.tolist()} lengths {counts[rows].tolist()}", flush=True)
        orc = oracle.Model(w.dims, w.J, R, np.ascontiguousarray(c[:, sel]), v[sel].astype(np.float64), A_now, B_now)
        orc.factor_pass(m, w.lr, w.lam)
        got = to_np(prm.A[m])[rows]
        want = orc.A[m][rows]
        before = A_now[m][rows]
        for k, i in enumerate(rows):
            ok, err, bound = delta_ok(got[k], want[k], before[k])
            assert ok, (m, int(i), int(counts[i]), err, bound)
        ft.refresh(plan, prm, m)


def test_relaxed_factor_passes_sampled_rows(netflix):
    """FT_RELAXED at full size (the plan of `bench.py --relaxed`): sampled rows against the oracle's
    relaxed module run on exactly their elements, from the same starting state."""
    import torch

    import paper_2210_06014_amd as ft

    w, c, v, A, B, _, _ = netflix
    J, R = w.J[0], w.R
    plan = ft.Plan(w.dims, J, R, c, v, relaxed=True)
    prm = ft.Params(A, B)
    ft.refresh(plan, prm)
    for m in range(3):
        A_now = [to_np(a) for a in prm.A]
        B_now = [to_np(b) for b in prm.B]
        ft.factor_pass(plan, prm, m, w.lr, w.lam)
        torch.cuda.synchronize()
        counts = np.bincount(c[m], minlength=w.dims[m])
        rows = _sample_rows(counts, plan, m)
        sel = np.isin(c[m], rows)
        print(f"[fullsize relaxed] mode {m}: rows {rows.tolist()} lengths {counts[rows].tolist()}", flush=True)
        orc = oracle.Model(w.dims, w.J, R, np.ascontiguousarray(c[:, sel]), v[sel].astype(np.float64), A_now, B_now)
        info = plan.mode_info(m)
        orc.factor_pass_relaxed(m, w.lr, w.lam, info["head"], info["chunk"])
        got = to_np(prm.A[m])[rows]
        want = orc.A[m][rows]
        before = A_now[m][rows]
        for k, i in enumerate(rows):
            ok, err, bound = delta_ok(got[k], want[k], before[k])
            assert ok, (m, int(i), int(counts[i]), err, bound)
        ft.refresh(plan, prm, m)
