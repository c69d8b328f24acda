"""Pins of the IC(0) oracle (Sec. 7.1's zero-fill incomplete Cholesky preconditioner).

Fixed points: where the pattern has no fill (a tridiagonal matrix with a tridiagonal
pattern, or the full pattern) IC(0) is the exact Cholesky factor of the library routine,
so PCG takes one iteration; on any pattern the product U^T U equals A on the pattern
(checked against brute-force entries), U vanishes off it, and U is upper triangular;
the stencil is symmetric and holds exactly (min(i+p,N) - max(i-p,0) + 1)^2 couplings for
an interior-row count (Sec. 3.1).
"""
import numpy as np
import pytest

from oracle import general, ic0
from paper_2105_01722_amd import inputs


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    return B @ B.T + n * np.eye(n)


def test_full_pattern_is_cholesky():
    A = _spd(12, 1)
    U = ic0.ic0(A, np.ones_like(A, dtype=bool))
    np.testing.assert_allclose(U, np.linalg.cholesky(A).T, rtol=1e-13, atol=1e-13)


def test_tridiagonal_has_no_fill():
    n = 15
    rng = np.random.default_rng(2)
    off = rng.uniform(-1, 1, n - 1)
    A = np.diag(3.0 + rng.uniform(0, 1, n)) + np.diag(off, 1) + np.diag(off, -1)
    P = np.abs(np.subtract.outer(np.arange(n), np.arange(n))) <= 1
    U = ic0.ic0(A, P)
    np.testing.assert_allclose(U, np.linalg.cholesky(A).T, rtol=1e-13, atol=1e-14)
    b = rng.standard_normal(n)
    x, its, _ = ic0.ic0_pcg(A, b, P, 1e-12, 50)
    assert its == 1
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-12)


def test_stencil_counts():
    N, p = 8, 3
    P = ic0.stencil(N, p)
    assert (P == P.T).all()
    w = np.array([min(k + p, N) - max(k - p, 0) + 1 for k in range(N + 1)])
    np.testing.assert_array_equal(P.sum(axis=1), np.outer(w, w).ravel())


@pytest.mark.parametrize("op", [0, 1])
def test_product_matches_on_pattern(op):
    """On an element matrix of a mapped element with variable c^2: U^T U = A entry by
    entry on the stencil (brute-force sums), U = 0 off it and below the diagonal."""
    N, p = 6, 3
    X, Y = inputs.node_coords(2, 2, N)
    c2 = inputs.c2_field(3, X, Y)
    X, Y = inputs.mapped_coords(X, Y)
    ops = general.GenOps(general.GenProblem(nx=2, ny=2, N=N, p=p), X, Y, c2)
    A = ic0.element_systems(ops, op)[1]
    P = ic0.stencil(N, p)
    U = ic0.ic0(A, P)
    n = A.shape[0]
    assert np.all(U[np.tril_indices(n, -1)] == 0.0)
    assert np.all(U[~P] == 0.0)
    for i in range(n):
        for j in range(i, n):
            if P[i, j]:
                s = sum(U[k, i] * U[k, j] for k in range(i + 1))
                assert abs(s - A[i, j]) <= 1e-12 * abs(A).max()
    # a dropped term would leave some pattern entry wrong; the preconditioned system is
    # then still close to the identity
    rng = np.random.default_rng(5)
    b = rng.standard_normal(n)
    x, its, _ = ic0.ic0_pcg(A, b, P, 1e-12, 200)
    assert 1 <= its <= 60
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10 * abs(x).max())


def test_breakdown_raises():
    A = np.array([[1.0, 2.0], [2.0, 1.0]])
    with pytest.raises(np.linalg.LinAlgError):
        ic0.ic0(A, np.ones((2, 2), dtype=bool))


def test_kronecker_mass_is_factored_exactly():
    """On a Cartesian element M_J = |Omega| Mref (x) Mref; the Cholesky factor of a Kronecker
    product is the Kronecker product of the factors, whose band stays inside the GD stencil,
    so IC(0) is exact and PCG on the dV/dt system takes one iteration (the paper's count of 1
    for dV/dt with its Kronecker mass matrix, Table 5)."""
    from oracle import gd1d
    N, p = 10, 3
    Mh, _ = gd1d.matrices_unit(N, p)
    Mref = Mh / N
    area = 0.37
    A = area * np.kron(Mref, Mref)
    U = ic0.ic0(A, ic0.stencil(N, p))
    Lr = np.linalg.cholesky(Mref)
    np.testing.assert_allclose(U, np.sqrt(area) * np.kron(Lr, Lr).T, rtol=1e-12,
                               atol=1e-13 * abs(U).max())
    b = np.random.default_rng(7).standard_normal(A.shape[0])
    _, its, _ = ic0.ic0_pcg(A, b, ic0.stencil(N, p), 1e-12, 10)
    assert its == 1
