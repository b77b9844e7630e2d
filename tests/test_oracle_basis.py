"""Pins of the oracle's LGL basis (Sec. 2.2) against closed forms and
library routines that share no code with it."""
import math
import os

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "lgl_closed_forms.txt")


def _closed_forms():
    rows = {}
    with open(GOLD) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            N, node, weight = line.split()
            env = {"sqrt": math.sqrt}
            rows.setdefault(int(N), []).append((eval(node, env), eval(weight, env)))
    return rows


def test_lgl_closed_forms(oracle_mod):
    for N, rows in _closed_forms().items():
        xi, w, _ = oracle_mod.lgl(N)
        np.testing.assert_allclose(xi, [r[0] for r in rows], rtol=0, atol=1e-15)
        np.testing.assert_allclose(w, [r[1] for r in rows], rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", range(1, 9))
def test_lgl_vs_numpy_legendre(oracle_mod, N):
    xi, w, _ = oracle_mod.lgl(N)
    # interior nodes = roots of P_N' (numpy's Legendre-series routines)
    c = np.zeros(N + 1); c[N] = 1.0
    roots = np.sort(npleg.legroots(npleg.legder(c))) if N > 1 else np.array([])
    np.testing.assert_allclose(xi[1:-1], roots, atol=2e-15)
    assert xi[0] == -1.0 and xi[-1] == 1.0
    # mirror symmetry is exact
    np.testing.assert_array_equal(xi, -xi[::-1])
    # quadrature: sum w = 2 and exactness for degree <= 2N-1
    assert abs(w.sum() - 2.0) < 1e-14
    for p in range(2 * N):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.dot(w, xi ** p) - exact) < 1e-14


@pytest.mark.parametrize("N", range(1, 9))
def test_derivative_matrix(oracle_mod, N):
    xi, w, D = oracle_mod.lgl(N)
    # D . 1 = 0
    assert np.abs(D.sum(axis=1)).max() < 1e-13 * N * N
    # exact differentiation of x^p for p <= N
    for p in range(N + 1):
        d = D @ xi ** p
        ex = p * xi ** (p - 1) if p > 0 else np.zeros_like(xi)
        assert np.abs(d - ex).max() < 1e-12 * (N + 1) ** 2
    # centro-antisymmetry D_{N-i,N-j} = -D_ij
    np.testing.assert_allclose(D[::-1, ::-1], -D, atol=1e-13 * N * N)
    # independent construction: barycentric differentiation matrix
    n1 = N + 1
    bw = np.array([1.0 / np.prod([xi[j] - xi[k] for k in range(n1) if k != j]) for j in range(n1)])
    Db = np.zeros((n1, n1))
    for i in range(n1):
        for j in range(n1):
            if i != j:
                Db[i, j] = bw[j] / bw[i] / (xi[i] - xi[j])
        Db[i, i] = -Db[i].sum()
    np.testing.assert_allclose(D, Db, atol=1e-12 * N * N)
    # summation-by-parts: W D + (W D)^T = diag(-1, 0, ..., 0, 1)
    Q = np.diag(w) @ D
    B = np.zeros((n1, n1)); B[0, 0] = -1.0; B[-1, -1] = 1.0
    np.testing.assert_allclose(Q + Q.T, B, atol=1e-13 * N * N)
