"""Default heads where the chain test of the plan's cost model binds: a tensor with few, long rows.

300 x 300 x 300 with 4M uniform elements (rows of about 13,300 elements, 300 per mode; J = R = 32).  The
quarter-of-elements row length alone would allow heads of 12288; the test that a head's serial chain end
within its launch cuts them to two chunks, so every row is a head plus a dozen chunk maps folded by the
combine.  Sampled rows of each mode's factor pass are checked against the oracle run on exactly their
elements, from the same starting state, with g shared per fiber (the default here) and per element.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import delta_ok, to_np

pytestmark = pytest.mark.gpu

DIMS, NNZ, J, R = [300, 300, 300], 4_000_000, 32, 32


@pytest.fixture(scope="module")
def problem():
    c, _ = synth.coords(DIMS, NNZ, 0.0, seed=21)
    v = synth.values(NNZ, "int1to5", seed=21)
    A, B = synth.init_params(DIMS, J, R, 0.1, seed=22)
    return c, v, A, B


def _rows(counts, head, chunk):
    order = np.argsort(-counts, kind="stable")
    picks = [order[0], order[len(order) // 2], order[-1]]
    for target in (head + 3 * chunk + 1, head + chunk):
        picks.append(int(np.argmin(np.abs(counts - target))))
    return np.unique(np.array(picks))


@pytest.mark.parametrize("fiber_share", [True, False])
def test_few_long_rows_default_heads(problem, fiber_share):
    import torch

    import paper_2210_06014_amd as ft

    c, v, A, B = problem
    print(f"\n[few rows] {DIMS} nnz={NNZ} J=R={J} fiber_share={fiber_share}", flush=True)
    plan = ft.Plan(DIMS, J, R, c, v, fiber_share=fiber_share)
    prm = ft.Params(A, B)
    ft.refresh(plan, prm)
    lr, lam = 1e-3, 1e-2
    for m in range(3):
        info = plan.mode_info(m)
        counts = np.bincount(c[m], minlength=DIMS[m])
        assert info["chunk"] == 1024 and info["head"] == 2048, info
        assert info["fiber_shared"] == int(fiber_share)
        assert counts.min() > info["head"] + 8 * info["chunk"]  # every row is a head and chunk maps
        A_now = [to_np(a) for a in prm.A]
        B_now = [to_np(b) for b in prm.B]
        ft.factor_pass(plan, prm, m, lr, lam)
        torch.cuda.synchronize()
        rows = _rows(counts, info["head"], info["chunk"])
        sel = np.isin(c[m], rows)
        print(f"[few rows] mode {m}: rows {rows.tolist()} lengths {counts[rows].tolist()}", flush=True)
        orc = oracle.Model(DIMS, [J] * 3, R, np.ascontiguousarray(c[:, sel]), v[sel].astype(np.float64), A_now, B_now)
        orc.factor_pass(m, lr, lam)
        got, want, before = to_np(prm.A[m])[rows], orc.A[m][rows], A_now[m][rows]
        for k, i in enumerate(rows):
            ok, err, bound = delta_ok(got[k], want[k], before[k])
            assert ok, (m, int(i), int(counts[i]), err, bound)
        ft.refresh(plan, prm, m)
