"""Writes tiny_epoch.json: the FP64 oracle's results for one small seeded problem (no value here comes from
the HIP path).  The paper prints no worked example with numbers (its FastTucker example is a figure), so
the stored values are the oracle's: one iteration of Algorithm 2 (factor module, then core module, Eq. (10),
(11)) and the loss of Eq. (6), plus one iteration with the relaxed factor module (head 8, chunk 4).

Run from the repository root: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

CASE = {"dims": [12, 9, 7], "nnz": 300, "zipf": 1.1, "J": 8, "R": 8, "sigma": 0.3, "seed": 77,
        "lr": 1e-2, "lam": 1e-2, "head": 8, "chunk": 4}


def inputs(case=CASE):
    c, _ = synth.coords(case["dims"], case["nnz"], case["zipf"], case["seed"])
    v = synth.values(case["nnz"], "int1to5", case["seed"])
    A, B = synth.init_params(case["dims"], case["J"], case["R"], case["sigma"], case["seed"] + 1)
    return c, v, A, B


def oracle_results(case=CASE):
    c, v, A, B = inputs(case)
    out = {}
    for kind in ("exact", "relaxed"):
        m = oracle.Model(case["dims"], case["J"], case["R"], c, v.astype(np.float64), [a.astype(np.float64) for a in A],
                         [b.astype(np.float64) for b in B])
        if kind == "exact":
            m.epoch(case["lr"], case["lam"], case["lr"], case["lam"])
        else:
            m.epoch_relaxed(case["lr"], case["lam"], case["lr"], case["lam"], case["head"], case["chunk"])
        out[kind] = {"A": [a.ravel().tolist() for a in m.A], "B": [b.ravel().tolist() for b in m.B],
                     "loss": m.loss(case["lam"], case["lam"]).tolist()}
    return out


if __name__ == "__main__":
    data = {"case": CASE, "source": "FP64 oracle (oracle/ft_oracle.c), written by tests/golden/make_golden.py",
            **oracle_results()}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_epoch.json"), "w") as f:
        json.dump(data, f, indent=0)
