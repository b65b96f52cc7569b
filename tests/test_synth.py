"""The seeded generator: distinct coordinates, draw-order prefix property, thread independence, law."""
import os
import subprocess
import sys

import numpy as np

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _keys(c, dims):
    k = np.zeros(c.shape[1], dtype=np.int64)
    for n, d in enumerate(dims):
        k = k * d + c[n]
    return k


def test_distinct_and_in_range():
    dims = [300, 200, 50]
    c, used = synth.coords(dims, 50_000, 1.1, seed=3)
    assert c.dtype == np.int32 and c.shape == (3, 50_000)
    for n, d in enumerate(dims):
        assert c[n].min() >= 0 and c[n].max() < d
    k = _keys(c, dims)
    assert len(np.unique(k)) == len(k)
    assert used >= 50_000


def test_prefix_property_and_determinism():
    """The first k coordinates do not depend on how many are asked for (first-drawn distinct are kept)."""
    dims = [100, 80, 60]
    c1, _ = synth.coords(dims, 20_000, 1.05, seed=9)
    c2, _ = synth.coords(dims, 60_000, 1.05, seed=9)
    np.testing.assert_array_equal(c1, c2[:, :20_000])
    c3, _ = synth.coords(dims, 20_000, 1.05, seed=10)
    assert not np.array_equal(c1, c3)


def test_thread_count_does_not_change_output():
    code = (
        "import sys; sys.path.insert(0, %r); import synth, numpy as np;"
        "c,u = synth.coords([1000, 700, 90], 300000, 1.1, 5); print(int(np.sum(c[0].astype(np.int64) * 7 + c[1] * 3 + c[2])), u)"
        % ROOT
    )
    outs = []
    for t in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env).strip())
    assert outs[0] == outs[1]


def test_zipf_marginal():
    """Draws follow P(k) ~ (k+1)^-s (before deduplication, which the sparse space makes negligible here)."""
    dims = [50, 10**6, 10**6]
    c, used = synth.coords(dims, 200_000, [1.2, 0.0, 0.0], seed=1)
    assert used == 200_000
    cnt = np.bincount(c[0], minlength=50).astype(np.float64)
    p = (np.arange(1, 51) ** -1.2)
    p /= p.sum()
    exp = p * 200_000
    chi2 = np.sum((cnt - exp) ** 2 / exp)
    assert chi2 < 100.0  # 49 degrees of freedom
    # uniform modes
    cu = np.bincount(c[1] // 100_000, minlength=10)
    assert np.all(np.abs(cu - 20_000) < 700)


def test_values_and_params():
    v = synth.values(100_000, "int1to5", seed=2)
    assert set(np.unique(v)) == {1.0, 2.0, 3.0, 4.0, 5.0}
    assert np.all(np.abs(np.bincount(v.astype(int))[1:] - 20_000) < 700)
    w = synth.values(100_000, "normal3", seed=2)
    assert w.min() >= 1.0 and w.max() <= 5.0 and abs(np.median(w) - 3.0) < 0.02
    A, B = synth.init_params([1000, 30], 8, 4, 0.1, seed=4)
    assert A[0].shape == (1000, 8) and B[1].shape == (8, 4) and A[0].dtype == np.float32
    assert abs(A[0].std() - 0.1) < 0.005 and abs(A[0].mean()) < 0.005
    A2, _ = synth.init_params([1000, 30], 8, 4, 0.1, seed=4)
    np.testing.assert_array_equal(A[0], A2[0])


def test_planted_values_and_split():
    """Planted values: seeded, in [1, 5], a separable signal with noise; the held-out split takes about 10 %."""
    dims = [500, 60, 7]
    c, _ = synth.coords(dims, 20_000, 1.1, seed=4)
    v1 = synth.planted(c, dims, seed=4)
    v2 = synth.planted(c, dims, seed=4)
    assert v1.dtype == np.float32 and np.array_equal(v1, v2)
    assert v1.min() >= 1.0 and v1.max() <= 5.0
    # without noise the values are 1 + 4 prod_n u_n with u_n in [0.3, 1)
    v0 = synth.planted(c, dims, seed=4, noise=0.0)
    assert v0.min() >= 1.0 + 4 * 0.3 ** 3 - 1e-5 and v0.max() < 5.0
    # the signal depends on the coordinates: equal coordinates give equal noiseless values
    order = np.lexsort(c[::-1])
    cs, vs = c[:, order], v0[order]
    same = np.all(cs[:, 1:] == cs[:, :-1], axis=0)
    assert np.all(vs[1:][same] == vs[:-1][same])
    m = synth.test_mask(200_000, seed=1)
    assert 0.09 < m.mean() < 0.11
