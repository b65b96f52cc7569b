"""Segment passes at a size where every wavefront walks several segments.

The core, loss, forward and gradient kernels give each wavefront a fixed set of segments (pieces of at most
512 elements of one row) and walk them trip by trip, loading the next segment's descriptor, C(m) row and
indices ahead, across segment boundaries.  Their grid holds at most 2048 workgroups of four wavefronts, so
a mode with more than 16384 segments makes every wavefront take at least two; these cases have 10M elements
and 20k-440k segments per mode (asserted).  The checks are the ones a dropped or repeated element at a
segment boundary would fail:

* forward: xhat of every element against the oracle, |d| <= 1e-5 sum_r prod_n |C(n)[i_n, r]|; the output
  is filled with NaN first, so an element the walk skips fails;
* loss: SSE against the oracle (rtol 1e-5) and against the FP64 sum of (x - xhat)^2 over the forward
  outputs (rtol 1e-9; the two kernels walk the same segments, and one element dropped or counted twice
  moves the SSE by about 1/|Omega| = 1e-7 of itself);
* gradient rows dA(n)[i] of every row against the oracle: ||d_i|| <= 1e-4 ||dA_i|| + 1e-7 max_i ||dA_i||
  (one element of a 250-element row is about 0.4 % of its row sum);
* core gradient (Eq. (11)): bit for bit -dB(n) of the gradient pass (the two launch the same grid and
  differ only in the sign of the residual), and within 1e-4 of the oracle's;
* one core pass per mode (Algorithm 5): B(n) row by row against the oracle's step.

BF16 storage: the Zipf case uses parameters BF16 holds exactly (A rounded to BF16, B(n) a diagonal of
signed powers of two, so C(n) = A(n) B(n) is exact in BF16 as in FP32); the BF16 kernels then read the
values the FP64 oracle uses and are held to the FP32 tolerances.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import abs_scale, to_np

pytestmark = pytest.mark.gpu

K_PARTIALS = 2048  # most workgroups a segment pass launches (four wavefronts each)

CASES = {
    # name: (dims, nnz, zipf, J, R, bf16-exact parameters)
    "uniform10M": ([40000, 40000, 40000], 10_000_000, 0.0, 16, 16, False),
    "zipf10M": ([480000, 18000, 2200], 10_000_000, 1.1, 16, 16, True),
}


def _bf16_exact_params(dims, J, R, seed):
    import torch

    assert J == R
    A, _ = synth.init_params(dims, J, R, 0.1, seed)
    A = [torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy() for a in A]
    rng = np.random.default_rng(seed)
    B = []
    for _ in dims:
        d = rng.choice([-1.0, 1.0], size=J) * np.exp2(-rng.integers(0, 3, size=J))
        B.append(np.diag(d).astype(np.float32))
    return A, B


@pytest.fixture(scope="module", params=list(CASES), ids=list(CASES))
def walk_case(request):
    import paper_2210_06014_amd as ft

    name = request.param
    dims, nnz, zipf, J, R, exact16 = CASES[name]
    print(f"\n[walk {name}] dims={dims} nnz={nnz} zipf={zipf} J={J} R={R}", flush=True)
    c, _ = synth.coords(dims, nnz, zipf, 31)
    v = synth.values(nnz, "int1to5", 31)
    if exact16:
        A, B = _bf16_exact_params(dims, J, R, 32)
    else:
        A, B = synth.init_params(dims, J, R, 0.1, 32)
    plan = ft.Plan(dims, J, R, c, v, with_perm=True)
    for m in range(len(dims)):
        segs = plan.mode_info(m)["segments"]
        print(f"[walk {name}] mode {m}: {segs} segments", flush=True)
        assert segs > 8 * K_PARTIALS, (m, segs)
    orc = oracle.Model(dims, J, R, c, v.astype(np.float64), [a.astype(np.float64) for a in A],
                       [b.astype(np.float64) for b in B])
    print(f"[walk {name}] oracle reference", flush=True)
    ref = {"xhat": orc.predict(c), "scale": abs_scale(orc.C, c), "loss": orc.loss()}
    ref["gA"], ref["gB"] = orc.grad()
    return name, dims, J, R, c, v, A, B, exact16, plan, orc, ref


def _storages(exact16):
    return ["f32", "bf16"] if exact16 else ["f32"]


def _params(walk_case, storage):
    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, exact16, plan, orc, ref = walk_case
    prm = ft.Params(A, B, storage=storage)
    ft.refresh(plan, prm)
    return prm


def test_forward_and_loss_walk(walk_case):
    name, dims, J, R, c, v, A, B, exact16, plan, orc, ref = walk_case
    for storage in _storages(exact16):
        _forward_and_loss(walk_case, storage)


def _forward_and_loss(walk_case, storage):
    import torch

    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, exact16, plan, orc, ref = walk_case
    prm = _params(walk_case, storage)
    out = torch.full((plan.nnz,), float("nan"), dtype=torch.float32, device="cuda")
    ft.forward(plan, prm, out=out)
    got = to_np(out)
    assert np.all(np.isfinite(got)), (name, storage, int(np.sum(~np.isfinite(got))))
    err = np.abs(got - ref["xhat"])
    bad = err > 1e-5 * ref["scale"] + 1e-30
    assert not bad.any(), (name, storage, int(bad.sum()), float(err.max()))
    sse = float(to_np(ft.loss(plan, prm))[0])
    host = float(np.sum((v.astype(np.float64) - got) ** 2))
    assert abs(sse - host) <= 1e-9 * host, (name, storage, sse, host)
    np.testing.assert_allclose(sse, ref["loss"][0], rtol=1e-5)


def test_gradient_rows_and_core_gradient_walk(walk_case):
    name, dims, J, R, c, v, A, B, exact16, plan, orc, ref = walk_case
    for storage in _storages(exact16):
        _gradient_rows(walk_case, storage)


def _gradient_rows(walk_case, storage):
    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, exact16, plan, orc, ref = walk_case
    prm = _params(walk_case, storage)
    gA, gB = ft.grad(plan, prm)
    for m in range(len(dims)):
        got = to_np(gA[m])
        want = ref["gA"][m]
        rows = np.flatnonzero(np.bincount(c[m], minlength=dims[m]))
        d = np.linalg.norm(got[rows] - want[rows], axis=1)
        nrm = np.linalg.norm(want[rows], axis=1)
        bound = 1e-4 * nrm + 1e-7 * nrm.max()
        worst = int(np.argmax(d / bound))
        assert np.all(d <= bound), (name, storage, m, int(rows[worst]), float(d[worst]), float(bound[worst]))
        # the core gradient of Algorithm 5 is -dB of 1/2 sum e^2, from the same walk
        G = to_np(ft.core_grad(plan, prm, m))
        dB = to_np(gB[m])
        assert np.array_equal(G, -dB), (name, storage, m, float(np.abs(G + dB).max()))
        Gr = -ref["gB"][m]
        assert np.linalg.norm(G - Gr) <= 1e-4 * np.linalg.norm(Gr), (name, storage, m)


def test_core_pass_walk(walk_case):
    """One core pass per mode from the same state, B(m) row by row against the oracle's step."""
    name, dims, J, R, c, v, A, B, exact16, plan, orc, ref = walk_case
    for storage in _storages(exact16):
        _core_pass(walk_case, storage)


def _core_pass(walk_case, storage):
    import torch

    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, exact16, plan, orc, ref = walk_case
    lr, lam = 1e-3, 1e-2
    for m in range(len(dims)):
        prm = _params(walk_case, storage)
        ft.core_pass(plan, prm, m, lr, lam)
        torch.cuda.synchronize()
        # the oracle's step from its own gradient: B + lr (G / |Omega| - lam B), G = -dB (Algorithm 5)
        B0 = orc.B[m]
        want = B0 + lr * (-ref["gB"][m] / plan.nnz - lam * B0)
        got = to_np(prm.B[m])
        for j in range(J):
            dj = np.linalg.norm(want[j] - B0[j])
            err = np.linalg.norm(got[j] - want[j])
            assert err <= 1e-3 * dj + 1e-6 * np.linalg.norm(want[j]), (name, storage, m, j, err, dj)


def test_run_reuse_matches_per_element_gathers(walk_case):
    """With FT_RUN_REUSE the segment passes gather the C row of mode m + 1 once per run of elements sharing
    it; the default walk gathers it for every element.  Both compute the same sums in a different order:
    loss, forward, gradient and core gradient agree to FP32 rounding, so the oracle checks of the default
    walk above carry over."""
    import paper_2210_06014_amd as ft

    name, dims, J, R, c, v, A, B, exact16, plan, orc, ref = walk_case
    reuse = ft.Plan(dims, J, R, c, v, with_perm=True, run_reuse=True)
    for m in range(len(dims)):
        assert reuse.mode_info(m)["runs"] < reuse.nnz
    for storage in _storages(exact16):
        got, base = {}, {}
        for tag, pl in (("reuse", reuse), ("plain", plan)):
            prm = _params((name, dims, J, R, c, v, A, B, exact16, pl, orc, ref), storage)
            out = {"loss": to_np(ft.loss(pl, prm)), "fwd": to_np(ft.forward(pl, prm))}
            gA, gB = ft.grad(pl, prm)
            for n in range(len(dims)):
                out[f"gA{n}"], out[f"gB{n}"] = to_np(gA[n]), to_np(gB[n])
                out[f"G{n}"] = to_np(ft.core_grad(pl, prm, n))
            (got if tag == "reuse" else base).update(out)
        np.testing.assert_allclose(got["loss"][:2], base["loss"][:2], rtol=1e-6)
        assert np.all(np.abs(got["fwd"] - base["fwd"]) <= 1e-6 * ref["scale"] + 1e-30), (name, storage)
        for n in range(len(dims)):
            for k in (f"gA{n}", f"gB{n}", f"G{n}"):
                d = np.linalg.norm(got[k] - base[k])
                assert d <= 1e-5 * np.linalg.norm(base[k]), (name, storage, k, d)
