"""Independent brute-force definitions used to pin the oracle on tiny tensors.

Nothing here calls the oracle.  The model is rebuilt from the paper's
definitions instead of its cached-intermediate formula:

* the Kruskal core  sum_r b(1)_r o ... o b(N)_r           (Definition 6)
* n-mode products with each A(n)                          (Definition 3, Eq. (1))
* matricization with the first remaining index fastest    (Definition 1)
* Kronecker and Khatri-Rao products                       (Definitions 7, 8)

and gradients are taken by central finite differences of the objective.
"""
from __future__ import annotations

import numpy as np


def kruskal_core(B):
    """Dense J_1 x ... x J_N core: sum over r of the outer products of the r-th columns."""
    R = B[0].shape[1]
    G = None
    for r in range(R):
        t = B[0][:, r]
        for n in range(1, len(B)):
            t = np.multiply.outer(t, B[n][:, r])
        G = t if G is None else G + t
    return G


def mode_product(X, M, n):
    """X x_n M for M of shape (I_n, J_n): contracts the J_n index of X with M's columns."""
    Y = np.tensordot(X, M, axes=([n], [1]))
    return np.moveaxis(Y, -1, n)


def dense_xhat(A, B):
    """Full reconstruction of Eq. (1): the Kruskal core multiplied by A(n) in every mode."""
    X = kruskal_core(B)
    for n, a in enumerate(A):
        X = mode_product(X, a, n)
    return X


def matricize(X, n):
    """X_(n): rows i_n, columns ordered with the lowest remaining mode fastest (Definition 1)."""
    I_n = X.shape[n]
    return np.moveaxis(X, n, 0).reshape(I_n, -1, order="F")


def kron_chain(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def khatri_rao(P, Q):
    """Column-wise Kronecker product: (P kr Q)[i*J + j, k] = P[i, k] Q[j, k]."""
    I, K = P.shape
    J, K2 = Q.shape
    assert K == K2
    return (P[:, None, :] * Q[None, :, :]).reshape(I * J, K)


def khatri_rao_chain(mats):
    out = mats[0]
    for m in mats[1:]:
        out = khatri_rao(out, m)
    return out


def matricized_xhat(A, B, n):
    """Eq. (3): X_(n) = A(n) B(n) Q^T S^T, S = A(N) kron .. (skip n) .. kron A(1), Q likewise with Khatri-Rao."""
    N = len(A)
    others = [k for k in range(N - 1, -1, -1) if k != n]
    S = kron_chain([A[k] for k in others])
    Q = khatri_rao_chain([B[k] for k in others])
    return A[n] @ B[n] @ Q.T @ S.T


def cells(X, coords):
    return X[tuple(coords[n] for n in range(coords.shape[0]))]


def half_sse(A, B, coords, vals, weights=None):
    """1/2 sum_x w_x (x - xhat_x)^2 with xhat from the dense reconstruction."""
    e = vals - cells(dense_xhat(A, B), coords)
    if weights is None:
        return 0.5 * float(np.sum(e * e))
    return 0.5 * float(np.sum(weights * e * e))


def central_fd(f, P, h=1e-3):
    """Central differences of f() w.r.t. every entry of P (restored after each probe).

    Every objective used here is quadratic in any single parameter entry (the model is multilinear),
    so central differences carry no truncation error; h only trades against rounding."""
    g = np.zeros_like(P)
    it = np.nditer(P, flags=["multi_index"])
    for _ in it:
        idx = it.multi_index
        old = P[idx]
        P[idx] = old + h
        fp = f()
        P[idx] = old - h
        fm = f()
        P[idx] = old
        g[idx] = (fp - fm) / (2 * h)
    return g


def cyclic_row_order(coords, m):
    """Elements grouped by i_m; within a row ordered by (i_{m+1}, ..., i_{m-1}) lexicographically."""
    N = coords.shape[0]
    keys = [coords[(m + k) % N] for k in range(N - 1, 0, -1)]  # least significant first for lexsort
    keys.append(coords[m])
    return np.lexsort(keys)


def sgd_factor_pass(A, B, coords, vals, m, lr, lam):
    """Row-major sequential SGD on A(m): each step moves a_{i_m} against the finite-difference gradient
    of f_x(a) = 1/2 (x - xhat_x)^2 + 1/2 lam ||a||^2 (gradient of Eq. (10)), other parameters fixed."""
    A = [a.copy() for a in A]
    for x in cyclic_row_order(coords, m):
        i = coords[m, x]
        c1 = coords[:, x : x + 1]
        v1 = vals[x : x + 1]
        row = A[m][i].copy()

        def f():
            A[m][i] = row
            return half_sse(A, B, c1, v1) + 0.5 * lam * float(row @ row)

        g = central_fd(f, row)
        A[m][i] = row - lr * g
    return A


def gd_core_pass(A, B, coords, vals, m, lr, lam):
    """One step on B(m) against the finite-difference gradient of
    1/2 mean_x (x - xhat_x)^2 + 1/2 lam ||B(m)||^2 (Eq. (11) summed over Omega, Algorithm 5)."""
    B = [b.copy() for b in B]
    nnz = coords.shape[1]
    Bm = B[m]

    def f():
        return half_sse(A, B, coords, vals) / nnz + 0.5 * lam * float(np.sum(Bm * Bm))

    g = central_fd(f, Bm)
    B[m] = Bm - lr * g
    return B
