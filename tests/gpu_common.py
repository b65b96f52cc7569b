"""Shared setup for the GPU parity tests: one seeded problem, fed to both the oracle and the HIP path."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def make_problem(dims, nnz, zipf, J, R, seed, sigma=0.1, values="int1to5"):
    c, _ = synth.coords(dims, nnz, zipf, seed)
    v = synth.values(nnz, values, seed)
    A, B = synth.init_params(dims, J, R, sigma, seed + 1)
    return c, v, A, B


def gpu_setup(dims, J, R, c, v, A, B, storage="f32", **plan_kw):
    import paper_2210_06014_amd as ft

    plan = ft.Plan(dims, J, R, c, v, **plan_kw)
    prm = ft.Params(A, B, storage=storage)
    ft.refresh(plan, prm)
    return plan, prm


def oracle_model(dims, J, R, c, v, A, B):
    return oracle.Model(dims, J, R, c, v.astype(np.float64), [a.astype(np.float64) for a in A],
                        [b.astype(np.float64) for b in B])


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def abs_scale(C_list, coords):
    """sum_r prod_n |C(n)[i_n, r]|: the natural scale of a rounding error in xhat."""
    p = None
    for n, C in enumerate(C_list):
        rows = np.abs(C[coords[n]])
        p = rows if p is None else p * rows
    return p.sum(axis=1)


def delta_ok(after_gpu, after_orc, before, rel=1e-3, abs_rel=1e-6):
    """Parity of one pass: ||gpu - oracle|| <= rel ||oracle - before|| + abs_rel ||oracle||, over the whole
    array and, for a matrix, over every row on its own, so that an error in one row's step (one element
    mishandled at a chunk, head or combine boundary) cannot hide among the other rows.  Returns
    (ok, err, bound) of the tightest of these checks (the largest err / bound)."""
    g, o, b = (np.asarray(x, dtype=np.float64) for x in (after_gpu, after_orc, before))
    err = [np.linalg.norm(g - o)]
    bound = [rel * np.linalg.norm(o - b) + abs_rel * np.linalg.norm(o)]
    if g.ndim == 2:
        err += list(np.linalg.norm(g - o, axis=1))
        bound += list(rel * np.linalg.norm(o - b, axis=1) + abs_rel * np.linalg.norm(o, axis=1))
    err, bound = np.array(err), np.array(bound)
    over = np.where(bound > 0, err / np.where(bound > 0, bound, 1.0), np.where(err > 0, np.inf, 0.0))
    k = int(np.argmax(over))
    return bool(np.all(err <= bound)), float(err[k]), float(bound[k])


def bf16_scale(A, B, coords):
    """sum_r prod_n S(n)[i_n, r] with S(n) = |A(n)| |B(n)|: the scale of BF16 rounding errors in xhat."""
    p = None
    for n in range(len(A)):
        S = np.abs(A[n].astype(np.float64)) @ np.abs(B[n].astype(np.float64))
        rows = S[coords[n]]
        p = rows if p is None else p * rows
    return p.sum(axis=1)
