"""One iteration of Algorithm 2 on the HIP path (exact and relaxed factor passes) against the stored oracle
results of tests/golden/tiny_epoch.json, from the same seeded inputs."""
import json
import os

import numpy as np
import pytest

from tests.gpu_common import delta_ok, gpu_setup, to_np
from tests.golden.make_golden import inputs

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("kind", ["exact", "relaxed"])
def test_gpu_matches_golden(kind):
    import paper_2210_06014_amd as ft

    stored = json.load(open(os.path.join(HERE, "tiny_epoch.json")))
    case = stored["case"]
    c, v, A, B = inputs(case)
    kw = {"chunk": case["chunk"], "head": case["head"]} if kind == "relaxed" else {}
    plan, prm = gpu_setup(case["dims"], case["J"], case["R"], c, v, A, B, relaxed=(kind == "relaxed"), **kw)
    ft.epoch(plan, prm, case["lr"], case["lam"], case["lr"], case["lam"])
    for n in range(len(case["dims"])):
        want = np.asarray(stored[kind]["A"][n]).reshape(A[n].shape)
        ok, err, bound = delta_ok(to_np(prm.A[n]), want, A[n].astype(np.float64))
        assert ok, (kind, "A", n, err, bound)
        want = np.asarray(stored[kind]["B"][n]).reshape(B[n].shape)
        ok, err, bound = delta_ok(to_np(prm.B[n]), want, B[n].astype(np.float64))
        assert ok, (kind, "B", n, err, bound)
    np.testing.assert_allclose(to_np(ft.loss(plan, prm, case["lam"], case["lam"])), stored[kind]["loss"], rtol=1e-4)
