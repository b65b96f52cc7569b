"""The RMSE and the parameters after 20 iterations of Algorithm 2 at full size, against the FP64 oracle.

tests/golden/make_fullsize_golden.py ran the oracle for 20 iterations on two full-size seeded workloads and
stored its training RMSE (and, for the planted tensor, its held-out RMSE) after every iteration, its B(n)
and sampled rows of its A(n) after the last one.  Here the HIP path runs the same 20 iterations from the
same inputs (the bench's default plan) and must reach:

* the final RMSE within 0.5 % of the oracle's (the contract's bound), in FP32 and with BF16 storage; the
  planted tensor is a regime where the RMSE falls from 2.16 to 0.26, so matching it says something;
* in FP32 the RMSE after every iteration within 1e-4 (measured on the planted tensor: 8e-6 at worst, in
  the steep descent; 4e-8 at the end).  With BF16 storage the curve runs slightly late or early during the
  steep descent (iterations 3-7 of the planted tensor, where one iteration moves the RMSE by 10-70 %):
  there a shift of a few hundredths of an iteration is a relative difference of a few percent (measured
  0.7-1.4 % at iteration 5, depending on the plan's piece lengths), so the bound before the last iteration
  is 5 %, which still catches a curve that stalls or diverges;
* in FP32, every sampled row of A(n) and every B(n) within 1e-4 of the distance the oracle moved it over the
  20 iterations (plus 1e-6 of its size), row by row (measured on the planted tensor: within 1e-5).  One
  element mishandled in a row's pass moves that row by about 1/L of its step (L its elements per pass), so
  the sampled short rows see such a mistake at once, and the longest rows see a lost chunk map.
"""
import json
import os

import numpy as np
import pytest

import synth
from tests.gpu_common import to_np

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RMSE_REL = 5e-3
F32_CURVE_REL = 1e-4
BF16_CURVE_REL = 5e-2
PARAM_REL = 1e-4


def _golden(name):
    path = os.path.join(GOLDEN, f"fullsize_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet (tests/golden/make_fullsize_golden.py {name})")
    with open(path) as f:
        return json.load(f)


def _trajectory(name, storage):
    import torch

    import paper_2210_06014_amd as ft

    g = _golden(name)
    w = synth.WORKLOADS[name]
    print(f"\n[fullsize golden] {name} {storage}: generating {w.nnz} elements", flush=True)
    c, v, A, B = synth.make(w)
    cte = vte = None
    if name == "planted":
        test = synth.test_mask(w.nnz, w.seed)
        cte = torch.from_numpy(np.ascontiguousarray(c[:, test])).cuda()
        vte = v[test].astype(np.float64)
        c, v = np.ascontiguousarray(c[:, ~test]), np.ascontiguousarray(v[~test])
    assert v.size == g["nnz_train"]
    plan = ft.Plan(w.dims, w.J[0], w.R, c, v)
    prm = ft.Params(A, B, storage=storage)
    ft.refresh(plan, prm)

    def rmse():
        tr = float(ft.loss(plan, prm)[1].item())
        te = None
        if cte is not None:
            err = ft.predict(plan, prm, cte).double().cpu().numpy() - vte
            te = float(np.sqrt(np.mean(err * err)))
        return tr, te

    train, test_ = [], []
    for it in range(g["iterations"] + 1):
        if it:
            ft.epoch(plan, prm, w.lr, w.lam, w.lr, w.lam)
        tr, te = rmse()
        train.append(tr)
        if te is not None:
            test_.append(te)
    torch.cuda.synchronize()
    return g, A, B, prm, np.array(train), np.array(test_)


def _check_curve(ref, got, label, what, curve_rel):
    ref = np.array(ref)
    rel = np.abs(got - ref) / ref
    print(f"[fullsize golden] {label}: {what} RMSE oracle {ref[-1]:.7f} gpu {got[-1]:.7f}, final relative "
          f"difference {rel[-1]:.2e}, largest {rel.max():.2e} (iteration {int(rel.argmax())})", flush=True)
    assert rel[-1] <= RMSE_REL, (label, what, "final", rel[-1])
    assert rel.max() <= curve_rel, (label, what, int(rel.argmax()), rel.max())


def _check_rmse(g, train, test_, label, curve_rel):
    _check_curve(g["train_rmse"], train, label, "train", curve_rel)
    if g["test_rmse"]:
        _check_curve(g["test_rmse"], test_, label, "held-out", curve_rel)


def _check_params(g, A0, B0, prm, label):
    worst = 0.0
    for n in range(len(A0)):
        rows = np.array(g["rows"][n])
        want = np.array(g["A_rows"][n])
        got = to_np(prm.A[n])[rows]
        before = A0[n][rows].astype(np.float64)
        err = np.linalg.norm(got - want, axis=1)
        bound = PARAM_REL * np.linalg.norm(want - before, axis=1) + 1e-6 * np.linalg.norm(want, axis=1)
        worst = max(worst, float(np.max(err / bound)))
        assert np.all(err <= bound), (label, n, rows[err > bound].tolist(), (err / bound).max())
        Bw = np.array(g["B"][n])
        eb = np.linalg.norm(to_np(prm.B[n]) - Bw)
        bb = PARAM_REL * np.linalg.norm(Bw - B0[n]) + 1e-6 * np.linalg.norm(Bw)
        worst = max(worst, eb / bb)
        assert eb <= bb, (label, n, eb, bb)
    print(f"[fullsize golden] {label}: parameters within {worst:.3f} of the bound", flush=True)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_planted_20_iterations(storage):
    g, A0, B0, prm, train, test_ = _trajectory("planted", storage)
    _check_rmse(g, train, test_, f"planted {storage}", F32_CURVE_REL if storage == "f32" else BF16_CURVE_REL)
    if storage == "f32":
        _check_params(g, A0, B0, prm, "planted f32")


def test_netflix_20_iterations():
    g, A0, B0, prm, train, test_ = _trajectory("netflix", "f32")
    _check_rmse(g, train, test_, "netflix f32", F32_CURVE_REL)
    _check_params(g, A0, B0, prm, "netflix f32")
