"""Host logic of the C-ABI library (no GPU): exported symbols, plan construction, error codes."""
import re
import os

import numpy as np
import pytest

import paper_2210_06014_amd as ft
import synth
from paper_2210_06014_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "fastertucker.h")).read()
    declared = set(re.findall(r"\b(ft_[a-z0-9_]+)\s*\(", header))
    assert declared == set(_lib.SYMBOLS)
    lib = _lib.load()
    for name in declared:
        assert hasattr(lib, name), name


def test_supported_table():
    assert ft.supported(3, 16, 16)
    assert ft.supported(3, 32, 32)
    assert ft.supported(8, 8, 16)
    assert not ft.supported(3, 12, 16)


def _plan(dims, J, R, coords, vals, **kw):
    return ft.Plan(dims, J, R, coords, vals, keep_host=True, upload=False, **kw)


@pytest.mark.parametrize("order", [3, 4, 8])
def test_run_counts(order):
    """The segment passes gather the C row of mode m + 1 once per run of a row's elements sharing that index;
    the plan's run count per mode is the number of (row, index of mode m + 1) changes along its sorted CSR,
    which for order 3 is the number of fibers of mode m + 2 (the elements with both fixed)."""
    dims = [40, 30, 20, 9, 8, 7, 6, 5][:order]
    c, _ = synth.coords(dims, 5000, 1.1, seed=9)
    v = synth.values(5000, "int1to5", seed=9)
    plan = _plan(dims, 8, 8 if order < 8 else 16, c, v)
    for m in range(order):
        row_ptr, idx, _, _ = plan.host_csr(m)
        rows = np.repeat(np.arange(dims[m]), np.diff(row_ptr))
        new = np.ones(c.shape[1], dtype=bool)
        new[1:] = (rows[1:] != rows[:-1]) | (idx[0][1:] != idx[0][:-1])
        assert plan.mode_info(m)["runs"] == int(new.sum()), m
        if order == 3:
            other = (m + 2) % 3
            pairs = {(int(a), int(b)) for a, b in zip(c[m], c[(m + 1) % 3])}
            assert len(pairs) == plan.mode_info(other)["fibers"] == int(new.sum())


@pytest.mark.parametrize("order", [3, 4])
def test_csr_order_and_permutation(order):
    dims = [37, 23, 11, 7][:order]
    J, R = (8, 8)
    c, _ = synth.coords(dims, 2000, 1.1, seed=5)
    v = synth.values(2000, "int1to5", seed=5)
    # duplicate a few coordinates: the plan must keep every element
    c = np.concatenate([c, c[:, :17]], axis=1)
    v = np.concatenate([v, v[:17] + 1])
    nnz = c.shape[1]
    chunk, head = 16, 40
    plan = _plan(dims, J, R, c, v, chunk=chunk, head=head)
    for m in range(order):
        row_ptr, idx, vals, perm = plan.host_csr(m)
        assert row_ptr[0] == 0 and row_ptr[-1] == nnz
        np.testing.assert_array_equal(np.diff(row_ptr), np.bincount(c[m], minlength=dims[m]))
        assert sorted(perm.tolist()) == list(range(nnz))
        np.testing.assert_array_equal(vals, v[perm])
        for k in range(order - 1):
            np.testing.assert_array_equal(idx[k], c[(m + 1 + k) % order][perm])
        # lexicographic (i_m, i_{m+1}, ..., i_{m-1}); ties keep input order (stable)
        keys = [c[(m + k) % order][perm] for k in range(order)]
        key_tuples = list(zip(*keys, perm))
        assert key_tuples == sorted(key_tuples)
        info = plan.mode_info(m)
        counts = np.diff(row_ptr)
        assert info["light_rows"] == int(np.sum((counts > 0) & (counts <= head)))
        assert info["heavy_rows"] == int(np.sum(counts > head))
        # a head plus ceil((L - head) / chunk) chunks per heavy row
        assert info["chunks"] == int(np.sum(np.where(counts > head, 1 + (counts - head + chunk - 1) // chunk, 0)))
        assert info["max_row"] == int(counts.max())


def test_errors():
    dims = [10, 10, 10]
    c, _ = synth.coords(dims, 100, 0.0, seed=1)
    v = np.ones(100, dtype=np.float32)
    bad = c.copy()
    bad[1, 57] = 10
    with pytest.raises(ft.FtError) as e:
        _plan(dims, 8, 8, bad, v)
    assert e.value.status == 3 and "element 57" in str(e.value)
    bad[1, 57] = -1
    with pytest.raises(ft.FtError) as e:
        _plan(dims, 8, 8, bad, v)
    assert e.value.status == 3
    with pytest.raises(ft.FtError) as e:
        _plan(dims, 12, 8, c, v)
    assert e.value.status == 4
    with pytest.raises(ft.FtError) as e:
        _plan(dims, [8, 8, 16], 8, c, v)
    assert e.value.status == 4
    with pytest.raises(ft.FtError) as e:
        _plan([10], 8, 8, c[:1], v)
    assert e.value.status == 2
    with pytest.raises(ft.FtError) as e:
        _plan([10, 0, 10], 8, 8, c, v)
    assert e.value.status == 2


def test_empty_tensor_plan():
    plan = _plan([5, 6, 7], 8, 8, np.zeros((3, 0), dtype=np.int32), np.zeros(0, dtype=np.float32))
    row_ptr, idx, vals, perm = plan.host_csr(0)
    assert row_ptr.sum() == 0 and idx.size == 0
    assert plan.mode_info(1)["nonempty_rows"] == 0


def test_calls_before_upload_fail_cleanly():
    c, _ = synth.coords([10, 10, 10], 50, 0.0, seed=1)
    plan = _plan([10, 10, 10], 8, 8, c, np.ones(50, dtype=np.float32))
    lib = _lib.load()
    st = lib.ft_factor_pass(plan.handle, None, 0, 1e-3, 1e-2, None)
    assert st == 5  # FT_ERR_STATE: not uploaded
    assert b"not uploaded" in lib.ft_last_error()


def test_fiber_counts():
    """Mode-m fibers (Section 3.2): distinct tuples of the other indices; shared when they hold >= 4 elements."""
    dims = [40, 30, 20]
    c, _ = synth.coords(dims, 6000, 1.2, seed=8)
    v = np.ones(c.shape[1], dtype=np.float32)
    plan = _plan(dims, 8, 8, c, v)
    for m in range(3):
        others = [n for n in range(3) if n != m]
        key = c[others[0]].astype(np.int64) * 100 + c[others[1]]
        nf = len(np.unique(key))
        info = plan.mode_info(m)
        assert info["fibers"] == nf
        assert info["fiber_shared"] == int(nf * 4 <= c.shape[1])
    off = ft.Plan(dims, 8, 8, c, v, keep_host=True, upload=False, fiber_share=False)
    assert all(off.mode_info(m)["fiber_shared"] == 0 for m in range(3))


def test_no_c_cache_flag():
    """FT_NO_C_CACHE: built for order 3 with J = R = 16; it turns fiber sharing off."""
    dims = [40, 30, 20]
    c, _ = synth.coords(dims, 6000, 1.2, seed=8)
    v = np.ones(c.shape[1], dtype=np.float32)
    plan = ft.Plan(dims, 16, 16, c, v, keep_host=True, upload=False, c_cache=False)
    assert all(plan.mode_info(m)["fiber_shared"] == 0 for m in range(3))
    for J, R, d in ((8, 8, dims), (32, 32, dims), (16, 16, dims + [5])):
        cc, _ = synth.coords(d, 500, 0.0, seed=3)
        with pytest.raises(ft.FtError) as e:
            ft.Plan(d, J, R, cc, np.ones(500, dtype=np.float32), keep_host=True, upload=False, c_cache=False)
        assert e.value.status == 4


def test_relaxed_flag():
    """FT_RELAXED keeps the plan's work lists as they are; it is refused with FT_NO_C_CACHE."""
    dims = [40, 30, 20]
    c, _ = synth.coords(dims, 6000, 1.2, seed=8)
    v = np.ones(c.shape[1], dtype=np.float32)
    exact = _plan(dims, 16, 16, c, v, chunk=16, head=40)
    relaxed = _plan(dims, 16, 16, c, v, chunk=16, head=40, relaxed=True)
    for m in range(3):
        assert exact.mode_info(m) == relaxed.mode_info(m)
        assert relaxed.mode_info(m)["heavy_rows"] > 0
    with pytest.raises(ft.FtError) as e:
        _plan(dims, 16, 16, c, v, relaxed=True, c_cache=False)
    assert e.value.status == 4


def test_relaxed_plan_deals_long_rows():
    """FT_RELAXED: in the order the factor passes read, a row longer than the head holds its sorted elements in
    stride order (Q = ceil(L / head): sorted positions 0, Q, 2Q, ..., then 1, 1 + Q, ...) in every per-element
    array; other rows keep the sorted order.  The arrays of the other passes stay sorted."""
    dims = [40, 30, 20]
    c, _ = synth.coords(dims, 6000, 1.2, seed=8)
    v = synth.values(c.shape[1], "int1to5", seed=8)
    head = 40
    exact = _plan(dims, 8, 8, c, v, chunk=16, head=head)
    relaxed = _plan(dims, 8, 8, c, v, chunk=16, head=head, relaxed=True)
    dealt_rows = 0
    for m in range(3):
        rp, idx, vals, perm = exact.host_csr(m)
        for a, b in zip(exact.host_csr(m, factor_order=True), relaxed.host_csr(m)):
            np.testing.assert_array_equal(a, b)
        rp2, idx2, vals2, perm2 = relaxed.host_csr(m, factor_order=True)
        np.testing.assert_array_equal(rp, rp2)
        for i in range(dims[m]):
            s, L = int(rp[i]), int(rp[i + 1] - rp[i])
            order = np.arange(L)
            if L > head:
                Q = -(-L // head)
                order = np.concatenate([np.arange(r, L, Q) for r in range(Q)])
                dealt_rows += 1
            np.testing.assert_array_equal(perm2[s:s + L], perm[s:s + L][order])
            np.testing.assert_array_equal(vals2[s:s + L], vals[s:s + L][order])
            np.testing.assert_array_equal(idx2[:, s:s + L], idx[:, s:s + L][:, order])
    assert dealt_rows > 0


def test_query_sizes_and_upload_refusals():
    """ft_plan_query: the plan's device arrays and the per-parameter-set scratch, known before upload;
    ft_plan_upload refuses a missing, short or misaligned workspace before it copies anything."""
    dims = [40, 30, 20]
    c, _ = synth.coords(dims, 6000, 1.2, seed=8)
    v = np.ones(c.shape[1], dtype=np.float32)
    J = R = 8
    plan = _plan(dims, J, R, c, v, chunk=16, head=40)
    nnz, N = c.shape[1], 3
    # every mode holds at least its row pointers, N - 1 index columns, values, segments and segment
    # pointers; the scratch at least the J x R partial sums of 2048 workgroups and the FP64 loss partials
    floor = sum(2 * (d + 1) * 8 + (N - 1) * nnz * 4 + nnz * 4 + plan.mode_info(m)["segments"] * 16
                for m, d in enumerate(dims))
    assert plan.device_bytes >= floor
    assert plan.scratch_bytes >= 2048 * J * R * 4 + 2048 * 8
    # sharing g per fiber adds the fiber arrays to the plan and the g table to the scratch
    shared = [m for m in range(3) if plan.mode_info(m)["fiber_shared"]]
    assert shared
    off = _plan(dims, J, R, c, v, chunk=16, head=40, fiber_share=False)
    assert plan.device_bytes - off.device_bytes >= sum(nnz * 4 for _ in shared)
    assert plan.scratch_bytes > off.scratch_bytes
    lib = _lib.load()
    fake = 1 << 20  # an aligned address the library must not touch: every case below fails before a copy
    for ptr, nbytes in ((None, plan.device_bytes), (fake, plan.device_bytes - 1), (fake + 8, plan.device_bytes)):
        assert lib.ft_plan_upload(plan.handle, ptr, nbytes, None) == 8  # FT_ERR_WORKSPACE
    assert lib.ft_plan_upload(None, fake, plan.device_bytes, None) == 1  # FT_ERR_ARG


def test_refuses_dims_beyond_32bit_gather_offsets():
    """C rows are gathered by 32-bit byte offsets: I_n * R * 4 must stay below 2^31 (FT_ERR_SHAPE)."""
    R = 32
    lim = (1 << 31) // (4 * R)
    c = np.zeros((3, 4), dtype=np.int32)
    v = np.ones(4, dtype=np.float32)
    for dims in ([lim, 5, 5], [5, 5, lim]):
        with pytest.raises(ft.FtError) as e:
            _plan(dims, R, R, c, v)
        assert e.value.status == 2
    ok = _plan([lim - 1, 5, 5], R, R, c, v)
    assert ok.mode_info(0)["rows"] == lim - 1


def _default_head(lens, chunk, J, shares_g):
    """The plan's default head of one mode, restated: the longest of 2..32 chunks (the listed counts), up to
    the cap (32 chunks at J >= 32, 24 at J = 16), not above L_q (the row length reached by the longest rows
    holding a quarter of the elements) and passing r_a h <= 0.8 (r_s S(h) + M(h))."""
    lens = np.sort(lens[lens > 0])[::-1].astype(np.int64)
    cs = np.cumsum(lens)
    lq = int(lens[min(np.searchsorted(4 * cs, cs[-1]), len(lens) - 1)])
    cap = chunk * (32 if J >= 32 else 24 if J >= 16 else 2)
    ra = (1200.0 if shares_g else 2358.0) if J >= 32 else (2000.0 if shares_g else 3100.0)
    rs = ((0.2 if J >= 32 else 0.3) if shares_g else 0.5)
    h = 2 * chunk
    for k in (3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32):
        c = k * chunk
        if c > cap or c > lq:
            break
        S = float(np.minimum(lens, c).sum())
        M = float(np.maximum(lens - c, 0).sum())
        if ra * min(c, int(lens[0])) > 0.8 * (rs * S + M):
            break
        h = c
    return h


def test_default_head_per_mode():
    """Exact plans pick each mode's head from its row lengths: the L_q bound binds on many rows of similar
    length, the chain bound on a few long rows, the cap on long Zipf rows; an explicit head and relaxed plans
    (two chunks) are kept as given."""
    J = R = 32
    # mode 0: 20 rows of about 20000 (chain bound); modes 1, 2: 2000 rows of about 200 (L_q bound)
    dims = [20, 2000, 2000]
    c, _ = synth.coords(dims, 400_000, 0.0, seed=11)
    v = synth.values(c.shape[1], "int1to5", seed=11)
    chunk = 16
    plan = _plan(dims, J, R, c, v, chunk=chunk)
    heads = []
    for m in range(3):
        info = plan.mode_info(m)
        lens = np.bincount(c[m], minlength=dims[m])
        assert info["chunk"] == chunk
        want = _default_head(lens, chunk, J, bool(info["fiber_shared"]))
        assert info["head"] == want, (m, info["head"], want)
        heads.append(info["head"])
    assert heads[0] < 20000 // 2 and heads[1] <= 200
    # Zipf rows, most elements in long rows: the cap (32 chunks at J = 32, 24 at J = 16) in modes 1 and 2
    dz = [20000, 50, 20]
    cz, _ = synth.coords(dz, 2_000_000, 1.3, seed=3)
    vz = synth.values(cz.shape[1], "int1to5", seed=3)
    for Jz, cap in ((32, 32), (16, 24)):
        pz = _plan(dz, Jz, Jz, cz, vz, chunk=16)
        for m in range(3):
            info = pz.mode_info(m)
            lens = np.bincount(cz[m], minlength=dz[m])
            assert info["head"] == _default_head(lens, 16, Jz, bool(info["fiber_shared"])), (Jz, m, info["head"])
        assert [pz.mode_info(m)["head"] for m in (1, 2)] == [cap * 16] * 2
    assert [_plan(dims, J, R, c, v, chunk=16, head=48).mode_info(m)["head"] for m in range(3)] == [48] * 3
    assert [_plan(dims, J, R, c, v, chunk=16, relaxed=True).mode_info(m)["head"] for m in range(3)] == [32] * 3
