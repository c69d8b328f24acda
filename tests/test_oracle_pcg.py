"""Pins of the PCG oracle (Sec. 7.1) and its tensor-product preconditioner.

Fixed points: on a Cartesian element with constant c^2 the preconditioner equals the
element matrix (simultaneous diagonalisation, Sec. 3.2), so PCG converges in one
iteration (cf. the single dV/dt iteration the paper reports for its Kronecker mass
matrix, Table 5); at any rtol the PCG solution matches a dense direct solve within
rtol * cond(A); iteration counts grow monotonically as rtol shrinks.
"""
import numpy as np
import pytest

from oracle import general, pcg
from paper_2105_01722_amd import inputs


def _ops(n=2, N=6, p=3, mapped=True, variable=True, flux="upwind", seed=3):
    X, Y = inputs.node_coords(n, n, N)
    c2 = inputs.c2_field(seed, X, Y) if variable else np.full_like(X, 1.3)
    if mapped:
        X, Y = inputs.mapped_coords(X, Y)
    return general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux=flux), X, Y, c2)


def _pmat(P, e, which, n1):
    cols = []
    for k in range(n1 * n1):
        r = np.zeros(n1 * n1)
        r[k] = 1.0
        cols.append(P.apply(e, r, which))
    return np.linalg.inv(np.array(cols).T)


def test_reference_eigenbasis():
    """Psi^T M_ref Psi = I, Psi^T S_ref Psi = diag(lam), lam_0 = 0, low modes ~ (k pi)^2."""
    from oracle import gd1d
    N, p = 16, 5
    Psi, lam = pcg.reference_eigenbasis(N, p)
    Mh, Sh = gd1d.matrices_unit(N, p)
    np.testing.assert_allclose(Psi.T @ (Mh / N) @ Psi, np.eye(N + 1), atol=1e-12)
    np.testing.assert_allclose(Psi.T @ (Sh * N) @ Psi, np.diag(lam), atol=1e-9 * lam.max())
    assert lam[0] == 0 and lam[1] > 0
    # Neumann Laplacian on [0, 1]: (k pi)^2
    np.testing.assert_allclose(lam[1:4], (np.arange(1, 4) * np.pi) ** 2, rtol=1e-5)


def test_preconditioner_exact_on_cartesian_constant():
    """Cartesian element, constant c^2: P_S = S_hat and P_M = M_J."""
    ops = _ops(n=2, N=6, p=3, mapped=False, variable=False)
    P = pcg.TensorPreconditioner(ops)
    n1 = ops.n1
    for e in range(4):
        np.testing.assert_allclose(_pmat(P, e, "S", n1), ops.Shat[e], atol=1e-9 * np.abs(ops.Shat[e]).max())
        np.testing.assert_allclose(_pmat(P, e, "M", n1), ops.M[e], atol=1e-12 * np.abs(ops.M[e]).max())


def test_mass_preconditioner_carries_the_mass_diagonal():
    """On mapped elements with a varying Jacobian the scaled mass preconditioner
    P_M = S^-1 Psi_2^-T diag(|Omega_k|) Psi_2^-1 S^-1 has exactly the diagonal of M_J (the
    property that defines the nodal scale s), stays symmetric positive definite, and is
    closer to M_J than the unscaled form (smaller spread of the eigenvalues of P_M^-1 M_J).
    A wrong index in s (ix and iy swapped, or the element's own area left out) breaks the
    diagonal identity on these elements, whose mapping is not symmetric in x and y."""
    X, Y = inputs.node_coords(2, 2, 8)
    Xm = X + 0.06 * np.sin(2 * np.pi * X) * np.cos(np.pi * Y)   # not symmetric in x and y
    Ym = Y + 0.02 * np.sin(2 * np.pi * Y)
    ops = general.GenOps(general.GenProblem(nx=2, ny=2, N=8, p=3, flux="upwind"), Xm, Ym,
                         inputs.c2_field(3, X, Y))
    P = pcg.TensorPreconditioner(ops)
    n1 = ops.n1
    s_saved = P.sM.copy()
    for e in range(4):
        PM = _pmat(P, e, "M", n1)
        np.testing.assert_allclose(np.diag(PM), np.diag(ops.M[e]), rtol=1e-12)
        np.testing.assert_allclose(PM, PM.T, atol=1e-13 * np.abs(PM).max())
        ev = np.linalg.eigvals(np.linalg.solve(PM, ops.M[e])).real
        P.sM[e] = 1.0
        ev0 = np.linalg.eigvals(np.linalg.solve(_pmat(P, e, "M", n1), ops.M[e])).real
        P.sM[e] = s_saved[e]
        assert ev.min() > 0 and ev.max() / ev.min() < ev0.max() / ev0.min()
    assert np.abs(s_saved - 1.0).max() > 1e-3     # the scale is not trivially one here


def test_one_iteration_when_exact():
    ops = _ops(n=2, N=6, p=3, mapped=False, variable=False)
    f = pcg.PcgRhs(ops, rtol=1e-13)
    rng = np.random.default_rng(0)
    U, V = rng.standard_normal((2, 2, 7, 7)), rng.standard_normal((2, 2, 7, 7))
    dU, dV = f(U, V)
    assert max(f.its_S[0]) <= 1 and max(f.its_M[0]) <= 1
    dU2, dV2 = general.rhs(U, V, ops)
    np.testing.assert_allclose(dU, dU2, atol=1e-11 * np.abs(dU2).max())


@pytest.mark.parametrize("rtol", [1e-6, 1e-10, 1e-14])
def test_pcg_matches_dense_within_conditioning(rtol):
    ops = _ops(n=2, N=7, p=5)
    f = pcg.PcgRhs(ops, rtol=rtol)
    rng = np.random.default_rng(1)
    U, V = rng.standard_normal((2, 2, 8, 8)), rng.standard_normal((2, 2, 8, 8))
    dU, dV = f(U, V)
    dU2, dV2 = general.rhs(U, V, ops)
    condS = max(np.linalg.cond(A) for A in ops.Shat)
    condM = max(np.linalg.cond(A) for A in ops.M)
    assert np.linalg.norm(dU - dU2) <= max(rtol * condS, 1e-13) * np.linalg.norm(dU2 - V) + 1e-13
    assert np.linalg.norm(dV - dV2) <= max(rtol * condM, 1e-13) * np.linalg.norm(dV2)
    assert max(f.its_S[0]) < 200 and max(f.its_M[0]) < 200


def test_iterations_monotone_in_rtol():
    ops = _ops(n=2, N=8, p=5)
    rng = np.random.default_rng(2)
    U, V = rng.standard_normal((2, 2, 9, 9)), rng.standard_normal((2, 2, 9, 9))
    prev = -1
    for rtol in (1e-2, 1e-6, 1e-10, 1e-14):
        f = pcg.PcgRhs(ops, rtol=rtol)
        f(U, V)
        tot = int(np.sum(f.its_S[0]) + np.sum(f.its_M[0]))
        assert tot >= prev
        prev = tot


def test_rk4_with_pcg_matches_dense():
    """A few RK4 steps with PCG (rtol 1e-14, warm starts) reproduce the dense-solve run."""
    ops = _ops(n=3, N=6, p=3)
    X, Y = inputs.node_coords(3, 3, 6)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=3), *inputs.mapped_coords(X, Y))
    V0 = np.zeros_like(U0)
    dt = 0.1 / 18
    f = pcg.PcgRhs(ops, rtol=1e-14)
    U1, V1 = general.run(U0, V0, ops, dt, 3, f=f)
    U2, V2 = general.run(U0, V0, ops, dt, 3)
    assert np.linalg.norm(U1 - U2) <= 1e-12 * np.linalg.norm(U2)
    assert np.linalg.norm(V1 - V2) <= 1e-11 * np.linalg.norm(V2)
    assert len(f.its_S) == 12
