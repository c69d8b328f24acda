"""Bloch (dispersion) analysis of the semi-discretisation -- FP64 oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 4: on a periodic grid of identical elements of width H the semi-discrete operator
commutes with the shift by one element, so its eigenvectors are Bloch waves: the state of
element e + 1 is exp(i theta) times that of element e.  Restricted to such a wave the
operator is the 2(N+1) x 2(N+1) symbol

    L(theta) = L_0 + exp(i theta) L_+ + exp(-i theta) L_-,

L_0 the coupling of an element's (u, v) to itself, L_+ / L_- to its east / west
neighbour, and its eigenvalues lambda = i Omega give the numerical dispersion relation
Omega(K) of all 2(N+1) modes at the wavenumber K = theta / H (one physical mode,
Omega ~ c K, and spurious ones).  The blocks are read from the oracle's right-hand side of
a y-independent strip of three elements (the invariant subspace used for the 1D rate
pins), assembled column by column.
"""
import numpy as np

from . import dg2d


def strip_blocks(N, p, flux, H=1.0, xi=1.0):
    """(L_-, L_0, L_+) of the 1D scheme on elements of width H, each 2(N+1) square, on
    z = (u, v) of one element (nodal values along x)."""
    n, n1 = 3, N + 1
    prob = dg2d.CartProblem(nx=n, ny=1, N=N, p=p, flux=flux, xi=xi, Lx=n * H, Ly=H)
    ops = dg2d.CartOps(prob)
    blocks = {d: np.zeros((2 * n1, 2 * n1)) for d in (-1, 0, 1)}
    for j in range(2 * n1):
        u = np.zeros((n, n1))
        v = np.zeros((n, n1))
        (u if j < n1 else v)[1, j % n1] = 1.0          # a unit state in element 1
        U = np.broadcast_to(u[None, :, None, :], (1, n, n1, n1)).copy()
        V = np.broadcast_to(v[None, :, None, :], (1, n, n1, n1)).copy()
        du, dv = dg2d.rhs(U, V, ops)
        for e, d in ((0, 1), (1, 0), (2, -1)):
            # the response of element e to element 1: element e sees element 1 as its
            # neighbour at offset d (d = +1: east neighbour)
            blocks[d][:, j] = np.concatenate([du[0, e, 0, :], dv[0, e, 0, :]])
    return blocks[-1], blocks[0], blocks[1]


def bloch_eigenvalues(N, p, flux, thetas, H=1.0, xi=1.0):
    """Eigenvalues of L(theta) for every theta (array [len(thetas), 2(N+1)], complex)."""
    Lm, L0, Lp = strip_blocks(N, p, flux, H, xi)
    return np.array([np.linalg.eigvals(L0 + np.exp(1j * t) * Lp + np.exp(-1j * t) * Lm)
                     for t in np.atleast_1d(thetas)])


def physical_mode(N, p, flux, K, H=1.0, xi=1.0):
    """The eigenvalue of the Bloch symbol nearest to i K (c = 1) for the wavenumber K,
    taken at theta = K H (K H must lie in (-pi, pi])."""
    lam = bloch_eigenvalues(N, p, flux, [K * H], H, xi)[0]
    return lam[np.argmin(np.abs(lam - 1j * K))]
