"""Pins of the oracle's relaxed factor module (chunks that read a long row as its head left it,
merged under a step guard).

The relaxed module is a reading of the unordered row updates of Algorithm 4,
not a formula the paper prints, so it is pinned by what its definition forces:
it is the serial pass of Algorithm 2 when no row is cut into chunks, it agrees
with the serial pass to second order in the learning rate, on a row whose
elements all share one g it follows the geometric closed form of SGD on a
single linear equation, guard included, and its head and chunks are the
residue classes of the stride deal, each equal to the serial pass over them.
"""
import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import _rng_params, _sparse


def _long_rows_problem(seed, dims=(3, 7, 6), nnz=90, J=3, R=4, scale=0.5):
    rng = np.random.default_rng(seed)
    Jl = [J] * len(dims)
    A, B = _rng_params(rng, dims, Jl, R, scale)
    coords, vals = _sparse(rng, dims, nnz)
    return dims, Jl, R, coords, vals, A, B


@pytest.mark.parametrize("m_mode", [0, 1, 2])
def test_relaxed_is_serial_without_chunks(m_mode):
    """head >= every row: the relaxed module is the factor module of Algorithm 2."""
    dims, J, R, c, v, A, B = _long_rows_problem(11)
    ser = oracle.Model(dims, J, R, c, v, A, B)
    rel = oracle.Model(dims, J, R, c, v, A, B)
    ser.factor_pass(m_mode, 0.05, 0.1)
    rel.factor_pass_relaxed(m_mode, 0.05, 0.1, head=1000, chunk=4)
    np.testing.assert_allclose(rel.A[m_mode], ser.A[m_mode], rtol=1e-13, atol=1e-15)


def test_one_chunk_from_the_start_is_serial():
    """head 0 and one chunk per row: the chunk starts from a0 and is the whole row, so the
    result is the serial one while the guard is inactive."""
    dims, J, R, c, v, A, B = _long_rows_problem(12)
    ser = oracle.Model(dims, J, R, c, v, A, B)
    rel = oracle.Model(dims, J, R, c, v, A, B)
    ser.factor_pass(0, 1e-3, 0.1)
    rel.factor_pass_relaxed(0, 1e-3, 0.1, head=0, chunk=1000)
    np.testing.assert_allclose(rel.A[0], ser.A[0], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("m_mode", [0, 2])
def test_second_order_agreement(m_mode):
    """Stale chunk reads change each step by O(lr) times the distance travelled since the
    start of the pass, itself O(lr): halving lr (lam fixed) quarters the difference to the
    serial pass.  A lost or misplaced decay factor would make it O(lr)."""
    dims, J, R, c, v, A, B = _long_rows_problem(13)
    diffs = []
    for lr in (4e-3, 2e-3, 1e-3):
        ser = oracle.Model(dims, J, R, c, v, A, B)
        rel = oracle.Model(dims, J, R, c, v, A, B)
        ser.factor_pass(m_mode, lr, 0.5)
        rel.factor_pass_relaxed(m_mode, lr, 0.5, head=2, chunk=3)
        moved = np.abs(ser.A[m_mode] - A[m_mode]).max()
        diffs.append(np.abs(rel.A[m_mode] - ser.A[m_mode]).max() / moved)
    # relative to the distance moved (O(lr)), the difference is O(lr): ratios near 2
    assert diffs[0] > 0
    for a, b in zip(diffs, diffs[1:]):
        assert 1.7 < a / b < 2.3, diffs


def _shared_g_row():
    """Mode 0 has one row; every element has the same g (all rows of A(1), A(2) equal) and the
    same value, so each step of a chunk is SGD on the single equation a.g = x."""
    dims, J, R = (1, 6, 5), [3, 3, 3], 4
    rng = np.random.default_rng(21)
    A0 = rng.normal(0, 0.5, size=(1, 3))
    A1 = np.repeat(rng.normal(0, 0.5, size=(1, 3)), 6, axis=0)
    A2 = np.repeat(rng.normal(0, 0.5, size=(1, 3)), 5, axis=0)
    B = [rng.normal(0, 0.7, size=(3, R)) for _ in range(3)]
    grid = np.stack(np.meshgrid(np.arange(1), np.arange(6), np.arange(5), indexing="ij")).reshape(3, -1)
    coords = grid.astype(np.int32)
    vals = np.full(coords.shape[1], 3.0)
    # g = B(0) w with w_r = C1[0, r] C2[0, r]
    w = (A1[0] @ B[1]) * (A2[0] @ B[2])
    g = B[0] @ w
    return dims, J, R, coords, vals, [A0, A1, A2], B, g


def _serial_shared_g(a, g, x, lr, lam, T):
    """T serial steps a <- rho a + lr (x - a.g) g with one fixed g, in closed form: the part of a
    orthogonal to g only decays, and u = a.g follows u <- p u + lr |g|^2 x with p = rho - lr |g|^2,
    a linear recurrence with fixed point u* = lr |g|^2 x / (1 - p)."""
    gg = g @ g
    rho = 1.0 - lr * lam
    p = rho - lr * gg
    u0 = a @ g
    ustar = lr * gg * x / (1.0 - p)
    uT = ustar + p ** T * (u0 - ustar)
    perp = a - (u0 / gg) * g
    return rho ** T * perp + (uT / gg) * g


@pytest.mark.parametrize("decay", [0.0, 0.02])
@pytest.mark.parametrize("step", [0.01, 0.5])
def test_shared_g_closed_form(step, decay):
    """On a row whose elements share g and x, T serial steps have the closed form above.  The
    head runs from a0 to a_H; chunk k (L_k elements) runs from a_H to b_k and contributes
    d_k = b_k - rho^{L_k} a_H, decayed by rho^{T_k} for the T_k elements after it; with
    omega = min(1, 1 / (lr (L - head) |g|^2)) the row becomes
    a_H + omega ((rho^{L - head} - 1) a_H + sum_k rho^{T_k} d_k).
    lr |g|^2 = 0.5 makes the guard act; lr lam = 0.02 weighs every chunk by its own decay."""
    dims, J, R, c, v, A, B, g = _shared_g_row()
    head, chunk = 4, 7
    L = c.shape[1]
    gg = g @ g
    lr = step / gg
    lam = decay / lr
    rho = 1.0 - lr * lam
    m = oracle.Model(dims, J, R, c, v, A, B)
    m.factor_pass_relaxed(0, lr, lam, head=head, chunk=chunk)
    a0 = A[0][0]
    a_head = _serial_shared_g(a0, g, 3.0, lr, lam, head)
    starts = list(range(head, L, chunk))
    lens = [min(chunk, L - s0) for s0 in starts]
    assert lens == [7, 7, 7, 5]
    S = sum(rho ** (L - s0 - Lk) * (_serial_shared_g(a_head, g, 3.0, lr, lam, Lk) - rho ** Lk * a_head)
            for s0, Lk in zip(starts, lens))
    omega = min(1.0, 1.0 / (step * (L - head)))
    assert (omega < 0.1) == (step == 0.5)
    want = a_head + omega * ((rho ** (L - head) - 1.0) * a_head + S)
    np.testing.assert_allclose(m.A[0][0], want, rtol=1e-12)
    if decay == 0.0:
        # chunk k moves the residual e_H by e_H (1 - q^{L_k}), q = 1 - lr |g|^2, and
        # omega sum_k (1 - q^{L_k}) <= omega lr |g|^2 (L - head) <= 1: the residual after the
        # pass lies between 0 and the residual after the head (no overshoot)
        e_head = 3.0 - a_head @ g
        e_after = 3.0 - m.A[0][0] @ g
        assert abs(e_after) <= abs(e_head) * (1 + 1e-12) and e_after * e_head >= 0


def test_guard_keeps_the_fixed_point():
    """The guard scales the whole merged step, decay included, so a row already at the balance of
    decay and data (here: a = 0 with x = 0) stays there, and rows damped by omega are not pulled
    towards zero faster than the data pulls them out: on the shared-g row with x = 3, lam > 0 and
    the guard active, a.g after the pass lies between its value after the head and the fixed point
    u* = lr |g|^2 x / (1 - rho + lr |g|^2) of the serial steps."""
    dims, J, R, c, v, A, B, g = _shared_g_row()
    gg = g @ g
    lr = 0.5 / gg
    lam = 0.02 / lr
    rho = 1.0 - lr * lam
    m = oracle.Model(dims, J, R, c, v, A, B)
    m.factor_pass_relaxed(0, lr, lam, head=4, chunk=7)
    u_head = _serial_shared_g(A[0][0], g, 3.0, lr, lam, 4) @ g
    u_star = lr * gg * 3.0 / (1.0 - rho + lr * gg)
    u_after = m.A[0][0] @ g
    lo, hi = sorted([u_head, u_star])
    assert lo - 1e-12 <= u_after <= hi + 1e-12, (u_head, u_after, u_star)


def test_decay_only_closed_form():
    """B(m) = 0 makes every g zero: each step only decays the row, and a row of L elements
    ends at (1 - lr lam)^L a0 whatever its head and chunks (the decay of the chunks is
    carried by the rho^{L - head} factor, their increments vanish)."""
    dims, J, R, c, v, A, B = _long_rows_problem(14)
    B = [b.copy() for b in B]
    B[0][:] = 0.0
    m = oracle.Model(dims, J, R, c, v, A, B)
    lr, lam = 0.1, 0.3
    m.factor_pass_relaxed(0, lr, lam, head=2, chunk=3)
    L = np.bincount(c[0], minlength=dims[0])
    want = A[0] * (1 - lr * lam) ** L[:, None]
    np.testing.assert_allclose(m.A[0], want, rtol=1e-13)


def test_long_rows_are_dealt_in_stride_order():
    """A row of L = 12 elements with head = chunk = 4 is dealt with stride Q = ceil(L / head) = 3: the head
    is the sorted positions 0, 3, 6, 9 and the two chunks are 1, 4, 7, 10 and 2, 5, 8, 11.  Each piece is run
    here by the serial module (pinned on its own) on exactly its elements, and merged as defined."""
    rng = np.random.default_rng(41)
    dims, J, R = (1, 4, 3), [3, 3, 3], 4
    A, B = _rng_params(rng, dims, J, R, 0.6)
    grid = np.stack(np.meshgrid(np.arange(1), np.arange(4), np.arange(3), indexing="ij")).reshape(3, -1)
    coords = grid.astype(np.int32)  # already in the row's sorted order (i_1, i_2)
    vals = rng.integers(1, 6, size=coords.shape[1]).astype(np.float64)
    lr, lam = 0.05, 0.1
    rho = 1.0 - lr * lam

    def serial(pos, start):
        m = oracle.Model(dims, J, R, coords[:, pos], vals[pos], [start[None, :], A[1], A[2]], B)
        m.factor_pass(0, lr, lam)
        return m.A[0][0]

    a_head = serial([0, 3, 6, 9], A[0][0])
    b1 = serial([1, 4, 7, 10], a_head)
    b2 = serial([2, 5, 8, 11], a_head)
    S = rho ** 4 * (b1 - rho ** 4 * a_head) + (b2 - rho ** 4 * a_head)
    C1, C2 = A[1] @ B[1], A[2] @ B[2]
    g = (C1[coords[1]] * C2[coords[2]]) @ B[0].T
    G = np.sum(g[[1, 4, 7, 10, 2, 5, 8, 11]] ** 2)
    omega = min(1.0, 1.0 / (lr * G))
    want = a_head + omega * ((rho ** 8 - 1.0) * a_head + S)
    m = oracle.Model(dims, J, R, coords, vals, A, B)
    m.factor_pass_relaxed(0, lr, lam, head=4, chunk=4)
    np.testing.assert_allclose(m.A[0][0], want, rtol=1e-12)
