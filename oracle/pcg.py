"""Preconditioned conjugate gradients for the element systems -- FP64 oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 7.1: for variable coefficients (and mapped elements) the element matrices of
DG1 / DG2 are inverted by preconditioned conjugate gradients.  The paper uses an
incomplete Cholesky preconditioner; here (a reading, not the paper's choice) the
preconditioner is the tensor-product operator of Sec. 3.2 built from element
averages:

  P_S = Psi_2^{-T} diag(D) Psi_2^{-1},  D_(ky,kx) = kbar_rr lam_kx + kbar_ss lam_ky,
        D_(0,0) = kappa |Omega_k|,
  P_M = S^-1 Psi_2^{-T} diag(|Omega_k|) Psi_2^{-1} S^-1,  S = diag(s),
        s_i = sqrt(|Omega_k| Mref_(iy,iy) Mref_(ix,ix) / (M_J)_ii),

with Psi, lam the simultaneous diagonalisation of the 1D GD stiffness and mass
matrices on the reference interval [0, 1] (Psi^T M_ref Psi = I), kbar_rr = int K_rr,
kbar_ss = int K_ss over the reference square, kappa the element-mean c^2 and
|Omega_k| = int J.  So P_S^{-1} r = Psi_2 diag(1/D) Psi_2^T r and
P_M^{-1} r = s o (Psi_2 Psi_2^T (s o r)) / |Omega_k|.  The nodal scale s gives P_M the
diagonal of M_J (Psi_2^{-T} Psi_2^{-1} = Mref (x) Mref, the reference mass), which follows
the Jacobian's variation inside the element.  On a Cartesian element with constant c^2,
P_S = S_hat and P_M = M_J exactly (s = 1; PCG converges in one iteration).

Stopping rule: ||r_k||_2 <= rtol ||b||_2 with r_k the CG recurrence residual
(r_0 = b - A x_0 computed directly, then r_{k+1} = r_k - alpha_k A d_k), at most maxit
iterations; x0 = the previous solution of the same element system (warm start), 0 at
the first call.  The paper does not say which residual it tests; the recurrence one
costs no extra product, and where it drifts from the true residual b - A x (about
eps cond(A) ||x|| at rtol near eps) the parity tests bound the result against the dense
direct solve instead.  ||b|| = 0 gives x = 0 with 0
iterations.  The S_hat system is solved for the correction y = dU/dt - V (right side
F_u), the M_J system for dV/dt.
"""
import numpy as np
import scipy.linalg as sla

from . import gd1d
from .general import lifts


def reference_eigenbasis(N, p):
    """Psi (columns = modes, Psi^T M_ref Psi = I) and lam of S_ref psi = lam M_ref psi on
    the reference interval [0, 1] (library generalised symmetric eigensolver)."""
    Mh, Sh = gd1d.matrices_unit(N, p)
    lam, Psi = sla.eigh(Sh * N, Mh / N)
    lam[0] = 0.0
    return Psi, lam


class TensorPreconditioner:
    """Element-wise D tables of P_S and P_M (plain), optionally scaled by exp(o)."""

    def __init__(self, ops, log_scale=None):
        prob = ops.prob
        self.n1 = n1 = prob.N + 1
        self.Psi, self.lam = reference_eigenbasis(prob.N, prob.p)
        ne = prob.nx * prob.ny
        D = (ops.kbar_rr[:, None, None] * self.lam[None, None, :]
             + ops.kbar_ss[:, None, None] * self.lam[None, :, None])       # [e, ky, kx]
        D[:, 0, 0] = ops.kappa * ops.area
        if log_scale is not None:
            o = np.asarray(log_scale, dtype=np.float64).reshape(ne, n1 * n1 - 1)
            Df = D.reshape(ne, -1)
            Df[:, 1:] *= np.exp(o)
            D = Df.reshape(ne, n1, n1)
        self.DS = D
        self.DM = ops.area.copy()
        Mh, _ = gd1d.matrices_unit(prob.N, prob.p)
        m = np.diag(Mh) / prob.N                     # diagonal of the reference mass on [0, 1]
        dPM = ops.area[:, None] * np.outer(m, m).ravel()[None, :]     # index iy*(N+1) + ix
        dMJ = np.stack([np.diag(ops.M[e]) for e in range(ne)])
        self.sM = np.sqrt(dPM / dMJ)

    def apply(self, e, r, which):
        """P^{-1} r for element e; r is a flat (N+1)^2 vector (index iy*(N+1) + ix)."""
        n1, Psi = self.n1, self.Psi
        if which == "M":
            r = self.sM[e] * r
        R = r.reshape(n1, n1)
        Rh = Psi.T @ R @ Psi                        # [ky, kx]
        Rh = Rh / (self.DS[e] if which == "S" else self.DM[e])
        z = (Psi @ Rh @ Psi.T).ravel()
        return self.sM[e] * z if which == "M" else z


def pcg(A, b, x0, apply_pinv, rtol, maxit):
    """Standard preconditioned CG (Hestenes-Stiefel form).  Returns (x, iterations)."""
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.zeros_like(b), 0
    x = x0.copy()
    r = b - A @ x
    if np.linalg.norm(r) <= rtol * nb:
        return x, 0
    z = apply_pinv(r)
    d = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = A @ d
        alpha = rz / (d @ q)
        x += alpha * d
        r -= alpha * q
        if np.linalg.norm(r) <= rtol * nb:
            return x, it
        z = apply_pinv(r)
        rz_new = r @ z
        d = z + (rz_new / rz) * d
        rz = rz_new
    return x, maxit


class PcgRhs:
    """Right-hand side of the general path with PCG element solves and warm starts.

    Call it as f(U, V) -> (dU/dt, dV/dt); iteration counts of every element solve are
    collected in `its_S`, `its_M` (one entry per call and element).
    """

    def __init__(self, ops, rtol=1e-12, maxit=200, log_scale=None):
        self.ops, self.rtol, self.maxit = ops, rtol, maxit
        self.P = TensorPreconditioner(ops, log_scale)
        ne = ops.prob.nx * ops.prob.ny
        nn = ops.n1 ** 2
        self.xS = np.zeros((ne, nn))
        self.xM = np.zeros((ne, nn))
        self.its_S, self.its_M = [], []

    def __call__(self, U, V):
        ops = self.ops
        prob = ops.prob
        ne = prob.nx * prob.ny
        Fu, Fv = lifts(U, V, ops)
        bS = Fu.reshape(ne, -1)
        bM = (-ops.apply_S(U) + Fv).reshape(ne, -1)
        itS, itM = np.zeros(ne, int), np.zeros(ne, int)
        for e in range(ne):
            self.xS[e], itS[e] = pcg(ops.Shat[e], bS[e], self.xS[e],
                                     lambda r: self.P.apply(e, r, "S"), self.rtol, self.maxit)
            self.xM[e], itM[e] = pcg(ops.M[e], bM[e], self.xM[e],
                                     lambda r: self.P.apply(e, r, "M"), self.rtol, self.maxit)
        self.its_S.append(itS)
        self.its_M.append(itM)
        return V + self.xS.reshape(U.shape), self.xM.reshape(U.shape).copy()
