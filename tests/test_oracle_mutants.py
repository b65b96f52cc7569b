"""Sensitivity of the oracle pins: each plausible mistake below, planted in a copy of the oracle's C file,
must make at least one pin fail.  CPU only: the copy is compiled with gcc and loaded by a pytest subprocess
that runs the pin files (FT_ORACLE_LIB points the oracle at it); the oracle itself is not modified."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ft_oracle.c")
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_relaxed.py"]

# (name, text of the oracle, replacement); every occurrence is replaced
MUTANTS = [
    ("sign of the data term in the factor step", "lr * (e * g[j] - lam * a[j])", "lr * (-e * g[j] - lam * a[j])"),
    ("decay dropped from the factor step", "lr * (e * g[j] - lam * a[j])", "lr * (e * g[j])"),
    ("core gradient not divided by |Omega|", "lr * (G[k] / (double)nnz - lam * Bm[k])", "lr * (G[k] - lam * Bm[k])"),
    ("core decay dropped", "lr * (G[k] / (double)nnz - lam * Bm[k])", "lr * (G[k] / (double)nnz)"),
    ("w includes the updated mode", "      if (n != m) p *= C[n][(int64_t)coords[n * nnz + x] * R + r];",
     "      p *= C[n][(int64_t)coords[n * nnz + x] * R + r];"),
    ("B read transposed in g", "s += Bm[(int64_t)j * R + r] * w[r];", "s += Bm[(int64_t)r * J + j] * w[r];"),
    ("fiber order: fixed indices compared from the last", "  for (int k = 1; k <= g_N; ++k) {\n    int n = (g_m + k) % g_N;",
     "  for (int k = g_N - 1; k >= 1; --k) {\n    int n = (g_m + k) % g_N;"),
    ("loss: sum of residuals instead of squares", "    sse += e * e;", "    sse += e;"),
    ("relaxed: chunk weight without the later decay", "decay_after = pow(rho, (double)(L - c1))", "decay_after = 1.0"),
    ("relaxed: guard off", "double omega = lr * G > 1.0 ? 1.0 / (lr * G) : 1.0;", "double omega = 1.0;"),
    ("relaxed: long rows not dealt in stride order", "    if (L > head && head > 0) {\n      int64_t Q",
     "    if (0) {\n      int64_t Q"),
    ("relaxed: guard on the increments only",
     "a[j] = a[j] + omega * ((decay_rest - 1.0) * a[j] + S[j]);", "a[j] = decay_rest * a[j] + omega * S[j];"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, name
    (tmp_path / "ft_oracle.c").write_text(src.replace(old, new))
    lib = str(tmp_path / "liborc.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", lib, str(tmp_path / "ft_oracle.c"), "-lm"])
    env = dict(os.environ, FT_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *PINS], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    # 1: some pin failed (a crash or a collection error would not show that the pins see the mistake)
    assert r.returncode == 1, (name, r.returncode, r.stdout[-2000:])
    assert "failed" in r.stdout, (name, r.stdout[-2000:])


def test_unmutated_oracle_passes_the_pins(tmp_path):
    lib = str(tmp_path / "liborc.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", lib, SRC, "-lm"])
    env = dict(os.environ, FT_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *PINS], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:]
