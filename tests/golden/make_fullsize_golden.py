"""Writes fullsize_<case>.json: the FP64 oracle's trajectory over 20 iterations of Algorithm 2 on a full-size
seeded workload (no value here comes from the HIP path), for the GPU test of the final RMSE after the same
iterations and of the parameters the iterations reach.

Cases:
  planted   the planted tensor (100000 x 10000 x 1000, 20M Zipf(1.1) coordinates, values of a separable model
            plus noise, 10 % held out; J = R = 16, init N(0, 0.3^2), lr = lam = 1e-2): a regime where the
            model learns, so matching the RMSE says something.
  netflix   the Netflix-shaped tensor (480000 x 18000 x 2200, 100M coordinates, values 1..5; J = R = 16,
            init N(0, 0.1^2), lr = 1e-3, lam = 1e-2) at the benchmark's hyperparameters.

Stored per iteration: the training RMSE (Eq. (6) without the regularisers) and, for the planted case, the
held-out RMSE.  After the last iteration: B(n) of every mode, and rows of A(n) (the longest rows of each mode
and a seeded sample of the others).  The oracle is single-threaded: the planted case takes about 20 minutes,
the netflix case a few hours.

Run from the repository root: python tests/golden/make_fullsize_golden.py planted|netflix
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

ITERS = 20
LONGEST = 8  # longest rows per mode
SAMPLED = 24  # further rows per mode, seeded uniform sample of the rows with elements


def case_inputs(name):
    """(workload, training coords, training values, held-out coords or None, held-out values or None, A0, B0)."""
    w = synth.WORKLOADS[name]
    c, v, A, B = synth.make(w)
    if name == "planted":
        test = synth.test_mask(w.nnz, w.seed)
        return (w, np.ascontiguousarray(c[:, ~test]), np.ascontiguousarray(v[~test]),
                np.ascontiguousarray(c[:, test]), v[test].astype(np.float64), A, B)
    return w, c, v, None, None, A, B


def sample_rows(coords, dims, seed):
    """Per mode: the LONGEST longest rows, then SAMPLED seeded rows among the other rows with elements."""
    rows = []
    for n, d in enumerate(dims):
        cnt = np.bincount(coords[n], minlength=d)
        longest = np.argsort(-cnt, kind="stable")[:LONGEST]
        rest = np.setdiff1d(np.nonzero(cnt)[0], longest)
        pick = synth.uniform_index(SAMPLED, rest.size, seed, 400 + n)
        rows.append(sorted(set(longest.tolist()) | set(rest[pick].tolist())))
    return rows


def main(name):
    w, c, v, cte, vte, A, B = case_inputs(name)
    dims = w.dims
    orc = oracle.Model(dims, w.J, w.R, c, v.astype(np.float64), [a.astype(np.float64) for a in A],
                       [b.astype(np.float64) for b in B])
    train, test = [float(orc.loss()[1])], []
    if cte is not None:
        test.append(float(np.sqrt(np.mean((orc.predict(cte) - vte) ** 2))))
    t0 = time.time()
    for it in range(ITERS):
        orc.epoch(w.lr, w.lam, w.lr, w.lam)
        train.append(float(orc.loss()[1]))
        if cte is not None:
            test.append(float(np.sqrt(np.mean((orc.predict(cte) - vte) ** 2))))
        print(f"[{name}] iteration {it + 1}: train RMSE {train[-1]:.9f}"
              + (f" test RMSE {test[-1]:.9f}" if test else "") + f" ({time.time() - t0:.0f} s)", flush=True)
    rows = sample_rows(c, dims, w.seed)
    data = {
        "case": name, "iterations": ITERS, "dims": dims, "nnz_train": int(v.size), "J": w.J[0], "R": w.R,
        "lr": w.lr, "lam": w.lam, "sigma": w.sigma, "seed": w.seed,
        "source": "FP64 oracle (oracle/ft_oracle.c), written by tests/golden/make_fullsize_golden.py",
        "train_rmse": train, "test_rmse": test,
        "rows": rows, "A_rows": [orc.A[n][rows[n]].tolist() for n in range(len(dims))],
        "B": [b.tolist() for b in orc.B],
        "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"fullsize_{name}.json")
    with open(path, "w") as f:
        json.dump(data, f)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
