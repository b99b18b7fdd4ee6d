"""Pins of the oracle's dense half (oracle/dense.c, oracle/gn.py): exact
integer cases, an error-free-transformation case, independent LAPACK routines
and the closed-form ridge solution of a linear least-squares problem.  CPU only."""
import numpy as np
import pytest

from oracle import dense
from oracle import gn as ogn


def test_gram_exact_on_integers_and_symmetric():
    rng = np.random.default_rng(1)
    J = rng.integers(-50, 50, size=(300, 40)).astype(np.float64)
    G = dense.gram(J)
    ref = (J.astype(np.int64).T @ J.astype(np.int64)).astype(np.float64)
    np.testing.assert_array_equal(G, ref)
    np.testing.assert_array_equal(G, G.T)


def test_gram_compensated_beats_naive_cancellation():
    # column products 1e16, 1, -1e16: naive FP64 summation loses the 1
    J = np.array([[1e16, 1e16], [1.0, 1.0], [-1e16, 1e16]])
    G = dense.gram(J)
    assert G[1, 0] == 1.0 and G[0, 1] == 1.0
    g = dense.gradient(J, np.array([1.0, 1.0, 1.0]))
    assert g[0] == 1.0


def test_gram_matches_blas_and_is_psd():
    rng = np.random.default_rng(2)
    J = rng.standard_normal((500, 60))
    G = dense.gram(J)
    assert np.linalg.norm(G - J.T @ J) / np.linalg.norm(G) < 1e-14
    assert np.linalg.eigvalsh(G).min() > -1e-12 * np.abs(G).max()
    rows = np.array([0, 5, 59, 10])
    cols = np.array([0, 3, 59, 10])
    np.testing.assert_array_equal(dense.gram_entries(J, rows, cols), G[rows, cols])


def test_cholesky_recovers_integer_factor_exactly():
    rng = np.random.default_rng(3)
    n = 30
    L0 = np.tril(rng.integers(-5, 6, size=(n, n))).astype(np.float64)
    L0[np.diag_indices(n)] = rng.integers(1, 6, size=n)
    A = L0 @ L0.T
    L, info = dense.cholesky(A)
    assert info == 0
    np.testing.assert_array_equal(L, L0)


def test_cholesky_reports_first_bad_pivot():
    A = np.diag([4.0, 1.0, -1.0, 2.0])
    _, info = dense.cholesky(A)
    assert info == 3
    B = np.array([[1.0, 2.0], [2.0, 4.0]])  # singular: second pivot is 0
    assert dense.cholesky(B)[1] == 2


def test_substitutions_against_lapack():
    rng = np.random.default_rng(4)
    n = 50
    L = np.tril(rng.standard_normal((n, n))) + 5 * np.eye(n)
    b = rng.standard_normal(n)
    np.testing.assert_allclose(dense.solve_lower(L, b), np.linalg.solve(L, b), rtol=1e-12)
    np.testing.assert_allclose(dense.solve_lower_t(L, b), np.linalg.solve(L.T, b), rtol=1e-12)
    A = L @ L.T
    np.testing.assert_allclose(dense.symv_lower(np.tril(A), b), A @ b, rtol=1e-13)


@pytest.mark.parametrize("mu", [1e-3, 1.0])
def test_one_step_is_exact_ridge_solution(mu):
    """r(theta) = A theta - b is linear in theta: one damped GN step lands on
    argmin |A theta - b|^2 + mu |theta - theta0|^2 (stacked least squares)."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((120, 35))
    b = rng.standard_normal(120)
    theta0 = rng.standard_normal(35)
    r = A @ theta0 - b
    G, g = ogn.gram_and_gradient(A, r)
    delta, info = ogn.damped_solve(G, g, mu)
    assert info == 0
    K = np.vstack([A, np.sqrt(mu) * np.eye(35)])
    rhs = np.concatenate([b, np.sqrt(mu) * theta0])
    ref = np.linalg.lstsq(K, rhs, rcond=None)[0]
    np.testing.assert_allclose(theta0 + delta, ref, rtol=1e-11, atol=1e-12)
    assert g @ delta < 0  # descent direction
    assert ogn.backward_error(G, mu, g, delta) < 1e-15


def test_damped_solve_reports_not_pd():
    G = np.diag([1.0, -2.0, 1.0])
    delta, info = ogn.damped_solve(G, np.ones(3), 0.5)
    assert delta is None and info == 2
