"""Pins of the 1D GD oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-runs the oracle's own
formula: the generating function is built here from eq. GD_basis_lagrange, the
matrices are checked against exact rational integration, textbook FEM values and
closed-form identities.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import gd1d


# ---------------------------------------------------------------------------
# independent helpers (exact rational polynomials, written for these tests)
# ---------------------------------------------------------------------------
def _lagrange_poly(nodes, a):
    """Coefficients (ascending, Fractions) of the Lagrange polynomial l_a on `nodes`."""
    coef = [Fraction(1)]
    for b, xb in enumerate(nodes):
        if b == a:
            continue
        den = Fraction(nodes[a] - xb)
        new = [Fraction(0)] * (len(coef) + 1)
        for k, c in enumerate(coef):
            new[k + 1] += c / den
            new[k] -= c * xb / den
        coef = new
    return coef


def _peval(c, t):
    return sum(float(ck) * t ** k for k, ck in enumerate(c))


def _pmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _pder(a):
    return [a[k] * k for k in range(1, len(a))] or [Fraction(0)]


def _pint(a, lo, hi):
    return sum(c * (Fraction(hi) ** (k + 1) - Fraction(lo) ** (k + 1)) / (k + 1)
               for k, c in enumerate(a))


def _Phi(p, x):
    """Generating function Phi_p of eq. GD_basis_lagrange (unit spacing), any real x.

    On [(q-j-1), (q-j)) (x >= 0) Phi_p = L_j, the Lagrange polynomial on G_j =
    {-j, ..., p-j} with L_j(0) = 1; Phi_p is even with support [-q, q].
    """
    q = (p + 1) // 2
    x = abs(x)
    if x >= q:
        return 0.0
    j = q - 1 - int(np.floor(x))
    nodes = list(range(-j, p - j + 1))
    return _peval(_lagrange_poly(nodes, nodes.index(0)), x)


# ---------------------------------------------------------------------------
def test_p3_ghost_closure_matches_worked_example():
    """Sec. 2.1.1, p = 3: u_{-1} = 4u0 - 6u1 + 4u2 - u3 and on (x0, x1)
    phi~0 = phi0 + 4 phi_{-1}, phi~1 = phi1 - 6 phi_{-1}, phi~2 = phi2 + 4 phi_{-1},
    phi~3 = phi3 - phi_{-1}; the oracle's cell-0 basis must equal these."""
    N, p = 8, 3
    coef = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden",
                                   "gd_p3_extrapolation_closure.txt"))[:, 1]
    t = np.linspace(0.0, 1.0, 23)[1:-1]
    phi, _ = gd1d.basis_on_cell(0, N, p, t)
    g = np.array([[_Phi(p, x - i) for i in range(-1, 4)] for x in t])  # phi_{-1..3}
    expect = np.stack([g[:, i + 1] + coef[i] * g[:, 0] for i in range(4)], axis=1)
    np.testing.assert_allclose(phi[:, :4], expect, atol=1e-14)
    np.testing.assert_array_equal(phi[:, 4:], 0.0)
    # the right boundary is the mirror image (Sec. 2.1.1 treats it the same way)
    phiR, _ = gd1d.basis_on_cell(N - 1, N, p, N - t)
    np.testing.assert_allclose(phiR[:, ::-1][:, :4], expect, atol=1e-14)


@pytest.mark.parametrize("p", [1, 3, 5, 7])
def test_interior_cells_match_generating_function(p):
    """Sec. 2.1, eq. GD_basis_lagrange: away from the boundary phi_i(x) = Phi_p(x - i)."""
    N = 3 * p + 4
    q = (p + 1) // 2
    t_loc = np.linspace(0.0, 1.0, 9)[:-1] + 0.03
    for k in range(N):
        if k - (q - 1) < 0 or k + q > N:
            continue  # closure cells
        phi, _ = gd1d.basis_on_cell(k, N, p, k + t_loc)
        ref = np.array([[_Phi(p, k + s - i) for i in range(N + 1)] for s in t_loc])
        np.testing.assert_allclose(phi, ref, atol=1e-13)


@pytest.mark.parametrize("p", [1, 3, 5, 7])
def test_generating_function_symmetric_compact(p):
    """Sec. 2.1: Phi_p(x) = Phi_p(-x), support [-q h, q h], Phi_p(0) = 1, zero at other nodes."""
    N = 4 * p + 6
    i = N // 2
    q = (p + 1) // 2
    s = np.linspace(-q - 1.5, q + 1.5, 97)
    phi, _ = gd1d.basis_eval(N, p, i + s)
    np.testing.assert_allclose(phi[:, i], phi[::-1, i], atol=1e-13)
    assert np.all(phi[np.abs(s) >= q, i] == 0.0)
    nodes, _ = gd1d.basis_eval(N, p, np.arange(N + 1, dtype=float))
    np.testing.assert_allclose(nodes, np.eye(N + 1), atol=1e-13)


@pytest.mark.parametrize("N,p", [(3, 3), (5, 3), (8, 3), (5, 5), (12, 5), (16, 5), (7, 7), (16, 7)])
def test_polynomial_reproduction_every_cell(N, p):
    """Nodal form (eq. GD_basis_nodalformula) with the closure reproduces x^m, m <= p,
    on every cell, boundary cells included (extrapolation of the interior order)."""
    t = np.concatenate([k + np.array([0.0, 0.17, 0.5, 0.83]) for k in range(N)] + [[float(N)]])
    phi, dphi = gd1d.basis_eval(N, p, t)
    xs = np.arange(N + 1, dtype=float)
    for m in range(p + 1):
        np.testing.assert_allclose(phi @ xs ** m, t ** m, rtol=1e-12, atol=1e-10)
        dm = m * t ** (m - 1) if m > 0 else np.zeros_like(t)
        np.testing.assert_allclose(dphi @ xs ** m, dm, rtol=1e-11, atol=1e-9)


def test_p1_is_linear_fem():
    """p = 1 is the hat function (Sec. 2.1): interior rows M = [1/6, 2/3, 1/6], S = [-1, 2, -1]."""
    N = 7
    M, S = gd1d.matrices_unit(N, 1)
    for i in range(1, N):
        np.testing.assert_allclose(M[i, i - 1:i + 2], [1 / 6, 2 / 3, 1 / 6], atol=1e-15)
        np.testing.assert_allclose(S[i, i - 1:i + 2], [-1, 2, -1], atol=1e-14)
    np.testing.assert_allclose([M[0, 0], S[0, 0]], [1 / 3, 1.0], atol=1e-15)


@pytest.mark.parametrize("N,p", [(6, 3), (9, 3), (8, 5), (12, 5), (16, 5), (9, 7), (16, 7)])
def test_matrix_identities(N, p):
    """Sec. 3.1: bandwidth p; S 1 = 0; S t = e_N - e_0 (int phi_i' = phi_i(N) - phi_i(0));
    1^T M 1 = N; t^T M 1 = N^2 / 2; both symmetric, M positive definite."""
    M, S = gd1d.matrices_unit(N, p)
    i, j = np.indices(M.shape)
    assert np.all(M[np.abs(i - j) > p] == 0) and np.all(S[np.abs(i - j) > p] == 0)
    one = np.ones(N + 1)
    t = np.arange(N + 1, dtype=float)
    np.testing.assert_allclose(S @ one, 0.0, atol=1e-12)
    e = np.zeros(N + 1)
    e[0], e[-1] = -1.0, 1.0
    np.testing.assert_allclose(S @ t, e, atol=1e-11)
    assert abs(one @ M @ one - N) < 1e-12
    assert abs(t @ M @ one - N * N / 2) < 1e-11
    np.testing.assert_allclose(M, M.T, atol=1e-15)
    np.testing.assert_allclose(S, S.T, atol=1e-13)
    assert np.linalg.eigvalsh(M).min() > 0


@pytest.mark.parametrize("N,p", [(3, 3), (6, 3), (5, 5), (8, 5)])
def test_gauss_assembly_equals_exact_rational(N, p):
    """The Gauss-rule assembly equals exact rational integration of the closure basis."""
    M, S = gd1d.matrices_unit(N, p)
    Me = [[Fraction(0)] * (N + 1) for _ in range(N + 1)]
    Se = [[Fraction(0)] * (N + 1) for _ in range(N + 1)]
    for k in range(N):
        s = min(max(k - (p - 1) // 2, 0), N - p)
        nodes = list(range(s, s + p + 1))
        L = [_lagrange_poly(nodes, a) for a in range(p + 1)]
        dL = [_pder(c) for c in L]
        for a in range(p + 1):
            for b in range(p + 1):
                Me[s + a][s + b] += _pint(_pmul(L[a], L[b]), k, k + 1)
                Se[s + a][s + b] += _pint(_pmul(dL[a], dL[b]), k, k + 1)
    np.testing.assert_allclose(M, np.array(Me, dtype=float), atol=1e-14)
    np.testing.assert_allclose(S, np.array(Se, dtype=float), atol=2e-13)


def test_face_vector_p3_one_sided_fd():
    """Sec. 3.2 D-tilde non-zeros: phi'(L) for p = 3 are the 4-point one-sided weights
    (-11/6, 3, -3/2, 1/3); phi'(R) is minus their mirror image; nnz = p + 1."""
    dL, dR = gd1d.face_vectors_unit(9, 3)
    np.testing.assert_allclose(dL[:4], [-11 / 6, 3, -3 / 2, 1 / 3], atol=1e-14)
    assert np.count_nonzero(dL) == 4 and np.count_nonzero(dR) == 4
    np.testing.assert_allclose(dR[::-1], -dL, atol=1e-14)


@pytest.mark.parametrize("N,p", [(5, 5), (12, 5), (16, 5), (7, 7), (16, 7), (8, 1)])
def test_face_vectors_exact_on_polynomials(N, p):
    """phi'(0) and phi'(N) differentiate every polynomial of degree <= p exactly."""
    dL, dR = gd1d.face_vectors_unit(N, p)
    t = np.arange(N + 1, dtype=float)
    for m in range(p + 1):
        assert abs(dL @ t ** m - (1.0 if m == 1 else 0.0)) < 1e-9 * max(1, N ** m)
        assert abs(dR @ t ** m - (m * N ** (m - 1) if m else 0.0)) < 1e-9 * max(1, N ** m)


def test_invalid_degree():
    with pytest.raises(ValueError):
        gd1d.matrices_unit(8, 4)
    with pytest.raises(ValueError):
        gd1d.matrices_unit(4, 5)
