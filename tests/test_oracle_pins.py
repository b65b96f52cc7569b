"""Pins of the FP64 oracle against the paper's definitions, closed forms and finite differences.

Each test checks the oracle against something other than itself: the dense
reconstruction of Eq. (1) built from Definitions 3 and 6, the matricized form
of Eq. (3), the textbook CP model, central finite differences of the
objective, and closed-form special cases of the update rules.
"""
import numpy as np
import pytest

import oracle
from tests import brute


def _rng_params(rng, dims, J, R, scale=0.5):
    A = [rng.normal(0, scale, size=(d, j)) for d, j in zip(dims, J)]
    B = [rng.normal(0, scale, size=(j, R)) for j in J]
    return A, B


def _all_coords(dims):
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    return np.stack([g.reshape(-1) for g in grids]).astype(np.int32)


def _sparse(rng, dims, nnz):
    full = _all_coords(dims)
    pick = rng.choice(full.shape[1], size=nnz, replace=False)
    coords = full[:, pick]
    vals = rng.integers(1, 6, size=nnz).astype(np.float64)
    return coords, vals


TINY = [((4, 5, 3), (2, 3, 2), 3), ((3, 4, 2, 3), (2, 2, 3, 2), 2), ((5, 3), (3, 2), 4)]


@pytest.mark.parametrize("dims,J,R", TINY)
def test_predict_equals_dense_reconstruction(dims, J, R):
    """Eq. (1) via n-mode products of the dense Kruskal core equals sum_r prod_n C(n)[i_n, r] (Eq. (12))."""
    rng = np.random.default_rng(1)
    A, B = _rng_params(rng, dims, J, R)
    coords = _all_coords(dims)
    m = oracle.Model(dims, J, R, coords, np.zeros(coords.shape[1]), A, B)
    got = m.predict(coords)
    want = brute.cells(brute.dense_xhat(A, B), coords)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("dims,J,R", TINY)
def test_predict_equals_matricized_form(dims, J, R):
    """Eq. (3): X_(n) = A(n) B(n) Q^T S^T with Kronecker S and Khatri-Rao Q, for every mode n."""
    rng = np.random.default_rng(2)
    A, B = _rng_params(rng, dims, J, R)
    coords = _all_coords(dims)
    m = oracle.Model(dims, J, R, coords, np.zeros(coords.shape[1]), A, B)
    X = np.zeros(dims)
    X[tuple(coords)] = m.predict(coords)
    for n in range(len(dims)):
        np.testing.assert_allclose(brute.matricize(X, n), brute.matricized_xhat(A, B, n), rtol=1e-12, atol=1e-14)


def test_cp_special_case():
    """J_n = R and B(n) = I reduce the model to the CP (Kruskal) model sum_r prod_n A(n)[i_n, r]."""
    rng = np.random.default_rng(3)
    dims, R = (4, 6, 5), 3
    A = [rng.normal(size=(d, R)) for d in dims]
    B = [np.eye(R) for _ in dims]
    coords = _all_coords(dims)
    m = oracle.Model(dims, R, R, coords, np.zeros(coords.shape[1]), A, B)
    cp = np.einsum("ir,jr,kr->ijk", *A)
    np.testing.assert_allclose(m.predict(coords), brute.cells(cp, coords), rtol=1e-12)


def test_rank_one_special_case():
    """R = 1: xhat = prod_n (a(n)_{i_n} . b(n))."""
    rng = np.random.default_rng(4)
    dims, J = (3, 4, 5), (2, 3, 2)
    A, B = _rng_params(rng, dims, J, 1)
    coords = _all_coords(dims)
    m = oracle.Model(dims, J, 1, coords, np.zeros(coords.shape[1]), A, B)
    want = np.ones(coords.shape[1])
    for n in range(3):
        want *= (A[n] @ B[n][:, 0])[coords[n]]
    np.testing.assert_allclose(m.predict(coords), want, rtol=1e-12)


def test_loss_against_dense():
    """Eq. (6): SSE, RMSE and the two regularisers, from the dense reconstruction and numpy norms."""
    rng = np.random.default_rng(5)
    dims, J, R = (5, 4, 6), (3, 2, 2), 3
    A, B = _rng_params(rng, dims, J, R)
    coords, vals = _sparse(rng, dims, 40)
    m = oracle.Model(dims, J, R, coords, vals, A, B)
    out = m.loss(0.3, 0.7)
    e = vals - brute.cells(brute.dense_xhat(A, B), coords)
    np.testing.assert_allclose(out[0], np.sum(e * e), rtol=1e-12)
    np.testing.assert_allclose(out[1], np.sqrt(np.mean(e * e)), rtol=1e-12)
    np.testing.assert_allclose(out[2], 0.3 * sum(np.sum(a * a) for a in A), rtol=1e-12)
    np.testing.assert_allclose(out[3], 0.7 * sum(np.sum(b * b) for b in B), rtol=1e-12)


@pytest.mark.parametrize("with_upstream", [False, True])
def test_gradient_finite_differences(with_upstream):
    """dA(n), dB(n) of Eq. (10)/(11) (no regularisers) equal central differences of the loss."""
    rng = np.random.default_rng(6)
    dims, J, R = (4, 5, 3), (2, 3, 2), 3
    A, B = _rng_params(rng, dims, J, R)
    coords, vals = _sparse(rng, dims, 25)
    m = oracle.Model(dims, J, R, coords, vals, A, B)
    if with_upstream:
        delta = rng.normal(size=coords.shape[1])

        def loss():
            return float(np.sum(delta * brute.cells(brute.dense_xhat(A, B), coords)))

        gA, gB = m.grad(delta)
    else:

        def loss():
            return brute.half_sse(A, B, coords, vals)

        gA, gB = m.grad()
    for n in range(3):
        fa = brute.central_fd(loss, A[n], h=1e-3)
        fb = brute.central_fd(loss, B[n], h=1e-3)
        np.testing.assert_allclose(gA[n], fa, rtol=1e-8, atol=1e-9)
        np.testing.assert_allclose(gB[n], fb, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("m_mode", [0, 1, 2])
def test_factor_pass_is_sequential_sgd(m_mode):
    """Factor module = per-element SGD steps (Eq. (9), (10)) in the canonical per-row order.

    The reference walks rows one after another with finite-difference gradients of the dense model,
    so it also checks that the oracle's fiber-major traversal equals row-major order."""
    rng = np.random.default_rng(7 + m_mode)
    dims, J, R = (4, 5, 3), (2, 3, 2), 3
    A, B = _rng_params(rng, dims, J, R, scale=0.6)
    coords, vals = _sparse(rng, dims, 30)
    lr, lam = 0.05, 0.1
    m = oracle.Model(dims, J, R, coords, vals, A, B)
    m.factor_pass(m_mode, lr, lam)
    want = brute.sgd_factor_pass(A, B, coords, vals, m_mode, lr, lam)
    for n in range(3):
        np.testing.assert_allclose(m.A[n], want[n], rtol=1e-8, atol=1e-10)
    np.testing.assert_array_equal(m.B[0], B[0])


@pytest.mark.parametrize("m_mode", [0, 1, 2])
def test_core_pass_is_gradient_step(m_mode):
    """Core module = one step on B(m) against the gradient of 1/2 mean e^2 + 1/2 lam ||B(m)||^2."""
    rng = np.random.default_rng(17 + m_mode)
    dims, J, R = (4, 5, 3), (2, 3, 2), 3
    A, B = _rng_params(rng, dims, J, R, scale=0.6)
    coords, vals = _sparse(rng, dims, 30)
    lr, lam = 0.3, 0.2
    m = oracle.Model(dims, J, R, coords, vals, A, B)
    m.core_pass(m_mode, lr, lam)
    want = brute.gd_core_pass(A, B, coords, vals, m_mode, lr, lam)
    for n in range(3):
        np.testing.assert_allclose(m.B[n], want[n], rtol=1e-8, atol=1e-10)


def test_epoch_matches_brute_force():
    """Algorithm 2: factor passes for modes 0..N-1, then core passes, every C(m) refreshed in between."""
    rng = np.random.default_rng(30)
    dims, J, R = (4, 3, 5), (2, 2, 3), 2
    A, B = _rng_params(rng, dims, J, R, scale=0.7)
    coords, vals = _sparse(rng, dims, 25)
    la, lama, lb, lamb = 0.04, 0.05, 0.2, 0.1
    m = oracle.Model(dims, J, R, coords, vals, A, B)
    m.epoch(la, lama, lb, lamb)
    A2, B2 = [a.copy() for a in A], [b.copy() for b in B]
    for n in range(3):
        A2 = brute.sgd_factor_pass(A2, B2, coords, vals, n, la, lama)
    for n in range(3):
        B2 = brute.gd_core_pass(A2, B2, coords, vals, n, lb, lamb)
    for n in range(3):
        np.testing.assert_allclose(m.A[n], A2[n], rtol=1e-8, atol=1e-10)
        np.testing.assert_allclose(m.B[n], B2[n], rtol=1e-8, atol=1e-10)
        np.testing.assert_allclose(m.C[n], A2[n] @ B2[n], rtol=1e-8, atol=1e-10)


def test_zero_learning_rate_is_noop():
    rng = np.random.default_rng(40)
    dims, J, R = (6, 5, 4), (3, 3, 3), 3
    A, B = _rng_params(rng, dims, J, R)
    coords, vals = _sparse(rng, dims, 60)
    m = oracle.Model(dims, J, R, coords, vals, A, B)
    m.epoch(0.0, 0.5, 0.0, 0.5)
    for n in range(3):
        np.testing.assert_array_equal(m.A[n], A[n])
        np.testing.assert_array_equal(m.B[n], B[n])


def test_decay_only_closed_form():
    """With C(k) = 0 for some k != m the shared g is 0, so each visit only decays: a <- (1 - lr lam)^count a."""
    rng = np.random.default_rng(41)
    dims, J, R = (6, 5, 4), (3, 3, 3), 3
    A, B = _rng_params(rng, dims, J, R)
    A[2][:] = 0.0
    coords, vals = _sparse(rng, dims, 70)
    lr, lam = 0.01, 0.3
    m = oracle.Model(dims, J, R, coords, vals, A, B)
    m.factor_pass(0, lr, lam)
    count = np.bincount(coords[0], minlength=dims[0])
    want = A[0] * ((1 - lr * lam) ** count)[:, None]
    np.testing.assert_allclose(m.A[0], want, rtol=1e-13)


def test_planted_model_is_fixed_point():
    """lam = 0 and x = xhat exactly: residuals vanish, so neither module moves the parameters."""
    rng = np.random.default_rng(42)
    dims, J, R = (6, 5, 4), (3, 2, 3), 3
    A, B = _rng_params(rng, dims, J, R)
    coords, _ = _sparse(rng, dims, 50)
    vals = brute.cells(brute.dense_xhat(A, B), coords)
    m = oracle.Model(dims, J, R, coords, vals, A, B)
    m.epoch(0.1, 0.0, 0.1, 0.0)
    for n in range(3):
        np.testing.assert_allclose(m.A[n], A[n], rtol=0, atol=1e-13)
        np.testing.assert_allclose(m.B[n], B[n], rtol=0, atol=1e-13)
    assert m.loss()[0] < 1e-24


def test_result_independent_of_input_order():
    """Only the per-row order matters; the oracle fixes it, so shuffling the input list changes nothing."""
    rng = np.random.default_rng(43)
    dims, J, R = (7, 6, 5), (3, 2, 2), 3
    A, B = _rng_params(rng, dims, J, R)
    coords, vals = _sparse(rng, dims, 90)
    perm = rng.permutation(coords.shape[1])
    m1 = oracle.Model(dims, J, R, coords, vals, A, B)
    m2 = oracle.Model(dims, J, R, coords[:, perm], vals[perm], A, B)
    m1.epoch(0.05, 0.1, 0.2, 0.1)
    m2.epoch(0.05, 0.1, 0.2, 0.1)
    for n in range(3):
        np.testing.assert_allclose(m1.A[n], m2.A[n], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(m1.B[n], m2.B[n], rtol=1e-12, atol=1e-14)


def test_row_order_matters():
    """Reversing the order of elements inside a row changes the factor pass (the steps do not commute)."""
    rng = np.random.default_rng(44)
    dims, J, R = (2, 6, 5), (2, 2, 2), 2
    A, B = _rng_params(rng, dims, J, R, scale=0.8)
    coords, vals = _sparse(rng, dims, 20)
    m = oracle.Model(dims, J, R, coords, vals, A, B)
    m.factor_pass(0, 0.2, 0.0)
    fwd = brute.sgd_factor_pass(A, B, coords, vals, 0, 0.2, 0.0)
    np.testing.assert_allclose(m.A[0], fwd[0], rtol=1e-8, atol=1e-10)
    # a different per-row order: the fixed indices in descending order
    order = brute.cyclic_row_order(coords, 0)[::-1]
    A3 = [a.copy() for a in A]
    for x in order:
        i = coords[0, x]
        row = A3[0][i].copy()
        c1, v1 = coords[:, x : x + 1], vals[x : x + 1]

        def f():
            A3[0][i] = row
            return brute.half_sse(A3, B, c1, v1)

        A3[0][i] = row - 0.2 * brute.central_fd(f, row)
    assert np.max(np.abs(A3[0] - m.A[0])) > 1e-6
