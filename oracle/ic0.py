"""Zero-fill incomplete Cholesky (IC(0)) of the element matrices -- FP64 oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 7.1 inverts the element matrices of DG1 / DG2 by preconditioned conjugate
gradients with an incomplete Cholesky preconditioner.  Its zero-fill form keeps the
sparsity of the matrix: the factor U (upper triangular, A ~ U^T U) may be nonzero only
where A's stencil is, and on that stencil U^T U reproduces A exactly.

Stencil (Sec. 3.1): two GD functions of degree p interact iff their 1D nodes are at
most p apart, so in 2D node (ix, iy) couples with (jx, jy) for |jx - ix| <= p and
|jy - iy| <= p; nodes are numbered i = iy (N + 1) + ix.  For S_hat = S_K + cw w w^T the
rank-one term is dense; the factor is taken of S_hat's entries on S_K's stencil (the
reading of the paper's IC(0) of the element matrix that keeps the factor sparse), while
the CG products use the whole S_hat.

The factor follows the definition of Cholesky with every entry off the stencil set to
zero: row by row, U_ii = sqrt(A_ii - sum_k<i U_ki^2) and
U_ij = (A_ij - sum_k<i U_ki U_kj) / U_ii on the stencil (j > i).  A non-positive pivot
is a breakdown and raises.
"""
import numpy as np
import scipy.linalg as sla

from .pcg import pcg


def stencil(N, p):
    """Boolean [nn, nn]: True where node i couples with node j (Sec. 3.1)."""
    n1 = N + 1
    ix = np.tile(np.arange(n1), n1)
    iy = np.repeat(np.arange(n1), n1)
    return (np.abs(ix[:, None] - ix[None, :]) <= p) & (np.abs(iy[:, None] - iy[None, :]) <= p)


def ic0(A, P):
    """Upper-triangular U with U_ij = 0 off the pattern P and (U^T U)_ij = A_ij on it."""
    n = A.shape[0]
    U = np.zeros_like(A, dtype=np.float64)
    for i in range(n):
        d = A[i, i] - U[:i, i] @ U[:i, i]
        if not d > 0.0:
            raise np.linalg.LinAlgError("IC(0) breakdown at row %d (pivot %r)" % (i, d))
        U[i, i] = np.sqrt(d)
        for j in range(i + 1, n):
            if P[i, j]:
                U[i, j] = (A[i, j] - U[:i, i] @ U[:i, j]) / U[i, i]
    return U


def ic0_apply(U):
    """r -> (U^T U)^{-1} r by the two triangular solves."""
    def f(r):
        y = sla.solve_triangular(U, r, trans="T", lower=False)
        return sla.solve_triangular(U, y, lower=False)
    return f


def element_systems(ops, op):
    """The element matrices of one kind for every element: op 0 is S_hat (the dU/dt
    system), op 1 is M_J (the dV/dt system)."""
    return ops.Shat if op == 0 else ops.M


def ic0_pcg(A, b, P, rtol, maxit):
    """IC(0)-preconditioned CG from x0 = 0 with the stop test of ``oracle.pcg.pcg``;
    returns (x, iterations, U)."""
    U = ic0(A, P)
    x, its = pcg(A, b, np.zeros_like(b), ic0_apply(U), rtol, maxit)
    return x, its, U
