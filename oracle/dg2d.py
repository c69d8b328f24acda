"""Energy-DG with a GD basis on a periodic Cartesian element grid, constant c -- oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain FP64, nodal state,
dense direct element solves.

Paper passages followed:
  * Sec. 2 eqs. eq:wave_1 / eq:wave_2: u_t = v, v_t = div(c^2 grad u) + f.
  * Sec. 2.1.2: 2D basis = tensor product of the modified 1D basis.
  * Sec. 2.2 eqs. DG1, DG2 and DG1_extra: the element-wise variational statement.
  * Sec. 2.2.1: numerical fluxes v*, (grad u)* with (alpha, beta, tau); central
    alpha = 1/2, beta = tau = 0; upwind alpha = 1/2, beta = xi/2, tau = 1/(2 xi).
  * Sec. 3.1: M = M_x (x) M_y, S = S_x (x) M_y + M_x (x) S_y.
  * Sec. 3.2: surface matrices are rank one: phi(X) phi(Y)^T and the like.
  * Sec. 3.3 / Sec. 6: classical fourth-order Runge-Kutta.

Readings (where the paper is silent, garbled or inconsistent):
  * The tau term of (grad u)* is read tau (v^1 n^1 + v^2 n^2) -- the only single-valued,
    dissipative reading.
  * The matrix forms DG_matrix1 / DG_matrix2 carry sign slips on the beta / tau face
    terms; the oracle is written from the variational form DG1 / DG2 instead.
  * The extra equation DG1_extra enters as S_hat = c^2 S + (kappa/|Omega_k|) w w^T with
    w_i = int phi_i and kappa = c^2; the solution y of S_hat y = F_u does not depend on
    kappa because 1^T F_u = 0.
  * Initial data is nodal interpolation (the paper's nodal formulation).
  * Physical boundaries (the paper states no boundary flux; its 2D Dirichlet experiment
    of Sec. 6 has homogeneous data): a wall face takes the interior flux formula with
    a mirror exterior state.  Dirichlet u = 0: the odd mirror, v_ext = -v and
    a_ext = -a (a = outward normal derivative); Neumann du/dn = 0: the even mirror,
    v_ext = v, a_ext = a.  With a GD basis that is symmetric under reflection this is
    exactly the periodic scheme on the domain doubled across the wall with odd (even)
    data, which is how it is pinned.
  * Source term: f(x, y, t) = sum_k sin(omega_k t + phase_k) g_k(x, y), each g_k
    represented by its GD interpolant (like the initial data), so the load vector of DG2
    is M g_k and the term adds sum_k sin(omega_k t + phase_k) g_k to dV/dt.  RK4 evaluates
    it at the stage times t, t + dt/2, t + dt/2, t + dt.

Array layout: a field on the element grid is [ny, nx, N+1 (iy), N+1 (ix)];
element (ex, ey) covers [x0 + ex Hx, x0 + (ex+1) Hx] x [y0 + ey Hy, ...];
node (ix, iy) sits at (x0 + ex Hx + ix hx, y0 + ey Hy + iy hy); nodes on faces are
duplicated per element.
"""
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import gd1d


def flux_params(flux, xi=1.0):
    """(alpha, beta, tau) of Sec. 2.2.1 for 'central', 'upwind' (xi: splitting speed) or
    'alternating' (alpha = 1, beta = tau = 0; the alpha of each face is face_alpha's)."""
    if flux == "central":
        return 0.5, 0.0, 0.0
    if flux == "upwind":
        return 0.5, 0.5 * xi, 0.5 / xi
    if flux == "alternating":
        return 1.0, 0.0, 0.0
    raise ValueError("flux must be 'central', 'upwind' or 'alternating'")


def face_alpha(flux, f, wall=False):
    """alpha on face f ("E", "W", "N", "S") of an element.

    Central and upwind: 1/2 on every face.  Alternating (Sec. 2.2.1 prints alpha = 1 with
    superscript 1 the inside of the element): taken literally every element would use its
    own v as v* on both sides of a face, a two-valued flux.  The reading used here fixes
    one orientation for each face: v* is the value of the element on the low-coordinate
    side (smaller x, or smaller y) and (grad u)* the gradient of the element on the high
    side.  Seen from an element that is alpha = 1 on its E and N faces and alpha = 0 on
    its W and S faces.  A wall face has no second element; there alpha = 1/2 (with
    beta = tau = 0 the mirror state then gives v* = 0 on a Dirichlet wall and
    n . (grad u)* = 0 on a Neumann wall, and the face exchanges no energy)."""
    if flux != "alternating" or wall:
        return 0.5
    return 1.0 if f in ("E", "N") else 0.0


@dataclass
class CartProblem:
    nx: int
    ny: int
    N: int
    p: int
    Lx: float = 1.0
    Ly: float = 1.0
    x0: float = 0.0
    y0: float = 0.0
    c2: float = 1.0
    flux: str = "central"
    xi: float = 1.0
    # boundary kind of the E, W, N, S sides: "periodic", "dirichlet" or "neumann"
    # (a direction is periodic on both of its sides or on neither)
    bc: tuple = ("periodic", "periodic", "periodic", "periodic")
    # source terms: tuple of (g_nodal [ny, nx, N+1, N+1], omega, phase)
    forcing: tuple = ()

    def __post_init__(self):
        kinds = ("periodic", "dirichlet", "neumann")
        bc = tuple(self.bc)
        if len(bc) != 4 or any(k not in kinds for k in bc):
            raise ValueError("bc: four of %s (E, W, N, S)" % (kinds,))
        for a, b in ((0, 1), (2, 3)):
            if (bc[a] == "periodic") != (bc[b] == "periodic"):
                raise ValueError("a direction is periodic on both sides or on neither")
        self.bc = bc

    @property
    def Hx(self):
        return self.Lx / self.nx

    @property
    def Hy(self):
        return self.Ly / self.ny

    @property
    def hx(self):
        return self.Hx / self.N

    @property
    def hy(self):
        return self.Hy / self.N


class CartOps:
    """1D and 2D element operators of one Cartesian element (Sec. 3.1, Sec. 3.2)."""

    def __init__(self, prob: CartProblem):
        gd1d.check_degree(prob.N, prob.p)
        self.prob = prob
        self.n1 = prob.N + 1
        self.Mx, self.Sx, self.dLx, self.dRx = gd1d.element_1d(prob.N, prob.p, prob.Hx)
        self.My, self.Sy, self.dLy, self.dRy = gd1d.element_1d(prob.N, prob.p, prob.Hy)
        # flattened element index = iy * n1 + ix, so an operator A_y on the y index and
        # B_x on the x index is kron(A_y, B_x)
        self.M2 = np.kron(self.My, self.Mx)
        self.S2 = np.kron(self.My, self.Sx) + np.kron(self.Sy, self.Mx)
        self.w = np.kron(self.My @ np.ones(self.n1), self.Mx @ np.ones(self.n1))
        area = prob.Hx * prob.Hy
        self.kappa = prob.c2
        self.Shat = prob.c2 * self.S2 + (self.kappa / area) * np.outer(self.w, self.w)
        self._chol_S = sla.cho_factor(self.Shat)
        self._chol_M = sla.cho_factor(self.M2)

    def solve_Shat(self, F):
        """Solve S_hat y = F for every element; F is [ny, nx, n1, n1]."""
        ny, nx, n1, _ = F.shape
        b = F.reshape(ny * nx, n1 * n1).T
        return sla.cho_solve(self._chol_S, b).T.reshape(F.shape)

    def solve_M(self, F):
        ny, nx, n1, _ = F.shape
        b = F.reshape(ny * nx, n1 * n1).T
        return sla.cho_solve(self._chol_M, b).T.reshape(F.shape)


def traces(U, V, ops):
    """Outward normal derivative a_f and value v_f on the four faces (Sec. 3.2 data).

    Returns dict f -> (a_f, v_f), each [ny, nx, n1] indexed by the position along the face.
    E: x = R, W: x = L, N: y = R, S: y = L.
    """
    aE = np.einsum("i,abji->abj", ops.dRx, U)
    aW = -np.einsum("i,abji->abj", ops.dLx, U)
    aN = np.einsum("j,abji->abi", ops.dRy, U)
    aS = -np.einsum("j,abji->abi", ops.dLy, U)
    return {
        "E": (aE, V[:, :, :, -1]),
        "W": (aW, V[:, :, :, 0]),
        "N": (aN, V[:, :, -1, :]),
        "S": (aS, V[:, :, 0, :]),
    }


# the elements on each side of the grid ([ny, nx, ...] indexing)
_SIDE = {"E": (slice(None), -1), "W": (slice(None), 0), "N": (-1, slice(None)),
         "S": (0, slice(None))}


def face_alphas(prob, f):
    """face_alpha of face f for every element, [ny, nx] (wall faces differ)."""
    al = np.full((prob.ny, prob.nx), face_alpha(prob.flux, f))
    if prob.bc["EWNS".index(f)] != "periodic":
        al[_SIDE[f]] = face_alpha(prob.flux, f, wall=True)
    return al


def neighbour_traces(tr, bc=("periodic",) * 4):
    """Traces of the neighbour across each face, on its opposite face: the periodic
    neighbour, or on a wall face the mirror state of the element's own traces
    (Dirichlet: a_ext = -a, v_ext = -v; Neumann: a_ext = a, v_ext = v)."""
    nb = {
        "E": tuple(np.roll(t, -1, axis=1) for t in tr["W"]),
        "W": tuple(np.roll(t, +1, axis=1) for t in tr["E"]),
        "N": tuple(np.roll(t, -1, axis=0) for t in tr["S"]),
        "S": tuple(np.roll(t, +1, axis=0) for t in tr["N"]),
    }
    for f, kind in zip("EWNS", bc):
        if kind == "periodic":
            continue
        sgn = -1.0 if kind == "dirichlet" else 1.0
        side = _SIDE[f]
        for k in (0, 1):
            nb[f][k][side] = sgn * tr[f][k][side]
    return nb


def face_sigmas(a, v, a_nb, v_nb, alpha, beta, tau):
    """sigma_u = v* - v^1 and sigma_v = n^1 . (grad u)* on one face (Sec. 2.2.1).

    With n^2 = -n^1, a = grad u^1 . n^1 and a_nb = grad u^2 . n^2:
      v*  - v^1       = (1 - alpha)(v^2 - v^1) - beta (a + a_nb)
      n^1 . (grad u)* = (1 - alpha) a - alpha a_nb + tau (v^2 - v^1)
    """
    jv = v_nb - v
    su = (1.0 - alpha) * jv - beta * (a + a_nb)
    sv = (1.0 - alpha) * a - alpha * a_nb + tau * jv
    return su, sv


def lifts(U, V, ops):
    """Face terms F_u, F_v of DG1 / DG2 for every element ([ny, nx, n1, n1] each).

    F_u,i = int_{dOmega} c^2 (n . grad phi_i) (v* - v) and F_v,i = int c^2 phi_i n.(grad u)*.
    On a face the traces are GD functions along the face with the nodal values of
    `traces`, so the face integrals are products with the 1D face mass matrix.
    """
    prob = ops.prob
    _, beta, tau = flux_params(prob.flux, prob.xi)
    c2 = prob.c2
    tr = traces(U, V, ops)
    nb = neighbour_traces(tr, prob.bc)
    sig = {f: face_sigmas(tr[f][0], tr[f][1], nb[f][0], nb[f][1],
                          face_alphas(prob, f)[:, :, None], beta, tau)
           for f in "EWNS"}
    Fu = np.zeros_like(U)
    Fv = np.zeros_like(V)
    # x-faces: normal derivative of phi_{ix,iy} is +-phi'_ix(R/L) phi_iy(y)
    mE_u = np.einsum("jk,abk->abj", ops.My, sig["E"][0])
    mW_u = np.einsum("jk,abk->abj", ops.My, sig["W"][0])
    mN_u = np.einsum("ik,abk->abi", ops.Mx, sig["N"][0])
    mS_u = np.einsum("ik,abk->abi", ops.Mx, sig["S"][0])
    Fu += c2 * np.einsum("i,abj->abji", ops.dRx, mE_u)
    Fu -= c2 * np.einsum("i,abj->abji", ops.dLx, mW_u)
    Fu += c2 * np.einsum("j,abi->abji", ops.dRy, mN_u)
    Fu -= c2 * np.einsum("j,abi->abji", ops.dLy, mS_u)
    Fv[:, :, :, -1] += c2 * np.einsum("jk,abk->abj", ops.My, sig["E"][1])
    Fv[:, :, :, 0] += c2 * np.einsum("jk,abk->abj", ops.My, sig["W"][1])
    Fv[:, :, -1, :] += c2 * np.einsum("ik,abk->abi", ops.Mx, sig["N"][1])
    Fv[:, :, 0, :] += c2 * np.einsum("ik,abk->abi", ops.Mx, sig["S"][1])
    return Fu, Fv


def apply_S2(U, ops):
    """(S_x (x) M_y + M_x (x) S_y) U for every element (Sec. 3.1)."""
    return (np.einsum("jl,ik,ablk->abji", ops.My, ops.Sx, U)
            + np.einsum("jl,ik,ablk->abji", ops.Sy, ops.Mx, U))


def rhs(U, V, ops, t=0.0):
    """Semi-discrete time derivatives (dU/dt, dV/dt) of DG1 + DG1_extra and DG2 at time t.

    S_hat (dU/dt - V) = F_u    and    M dV/dt = -c^2 S U + F_v + sum_k s_k(t) M g_k.
    """
    Fu, Fv = lifts(U, V, ops)
    y = ops.solve_Shat(Fu)
    z = ops.solve_M(-ops.prob.c2 * apply_S2(U, ops) + Fv)
    return V + y, z + forcing_term(ops.prob, t)


def forcing_term(prob, t):
    """sum_k sin(omega_k t + phase_k) g_k (nodal; zero without source terms)."""
    out = 0.0
    for g, omega, phase in prob.forcing:
        out = out + np.sin(omega * t + phase) * np.asarray(g, dtype=np.float64)
    return out


def rk4_step(U, V, dt, f):
    """One classical RK4 step for Z' = f(Z), Z = (U, V)."""
    k1u, k1v = f(U, V)
    k2u, k2v = f(U + 0.5 * dt * k1u, V + 0.5 * dt * k1v)
    k3u, k3v = f(U + 0.5 * dt * k2u, V + 0.5 * dt * k2v)
    k4u, k4v = f(U + dt * k3u, V + dt * k3v)
    return (U + dt / 6.0 * (k1u + 2 * k2u + 2 * k3u + k4u),
            V + dt / 6.0 * (k1v + 2 * k2v + 2 * k3v + k4v))


def rk4_step_t(U, V, t, dt, f):
    """One classical RK4 step for Z' = f(t, Z) from time t."""
    k1u, k1v = f(t, U, V)
    k2u, k2v = f(t + 0.5 * dt, U + 0.5 * dt * k1u, V + 0.5 * dt * k1v)
    k3u, k3v = f(t + 0.5 * dt, U + 0.5 * dt * k2u, V + 0.5 * dt * k2v)
    k4u, k4v = f(t + dt, U + dt * k3u, V + dt * k3v)
    return (U + dt / 6.0 * (k1u + 2 * k2u + 2 * k3u + k4u),
            V + dt / 6.0 * (k1v + 2 * k2v + 2 * k3v + k4v))


def run(U, V, ops, dt, steps, t0=0.0):
    """steps RK4 steps from time t0 (the time only enters through source terms)."""
    if not ops.prob.forcing:
        for _ in range(steps):
            U, V = rk4_step(U, V, dt, lambda a, b: rhs(a, b, ops))
        return U, V
    for s in range(steps):
        U, V = rk4_step_t(U, V, t0 + s * dt, dt, lambda t, a, b: rhs(a, b, ops, t))
    return U, V


def energy(U, V, ops):
    """Discrete energy sum_k 1/2 V^T M V + 1/2 c^2 U^T S U (Sec. 2.2, the energy that
    DG1 / DG2 conserve under the central flux)."""
    ny, nx, n1, _ = U.shape
    u = U.reshape(ny * nx, n1 * n1)
    v = V.reshape(ny * nx, n1 * n1)
    eu = np.einsum("ei,ij,ej->", u, ops.S2, u)
    ev = np.einsum("ei,ij,ej->", v, ops.M2, v)
    return 0.5 * ev + 0.5 * ops.prob.c2 * eu


def energy_rate(U, V, ops):
    """dE/dt of the semi-discretisation = sum_k (U^T F_u + V^T F_v) (from DG1, DG2)."""
    Fu, Fv = lifts(U, V, ops)
    return float(np.sum(U * Fu) + np.sum(V * Fv))


def node_coords(prob):
    """Physical node coordinates X, Y, each [ny, nx, n1, n1] (the layout above)."""
    n1 = prob.N + 1
    ex = np.arange(prob.nx)
    ey = np.arange(prob.ny)
    i = np.arange(n1)
    X = prob.x0 + ex[None, :, None, None] * prob.Hx + i[None, None, None, :] * prob.hx
    Y = prob.y0 + ey[:, None, None, None] * prob.Hy + i[None, None, :, None] * prob.hy
    X = np.broadcast_to(X, (prob.ny, prob.nx, n1, n1)).copy()
    Y = np.broadcast_to(Y, (prob.ny, prob.nx, n1, n1)).copy()
    return X, Y


def l2_error(U, prob, exact, nq=None):
    """||u_h - u|| in L^2 over the domain by Gauss quadrature of the GD interpolant
    (Sec. 6 error measure).  `exact(x, y)` is vectorised."""
    N, p = prob.N, prob.p
    nq = nq or (p + 3)
    xg, wg = gd1d.gauss_legendre(nq)
    tq = (np.arange(N)[:, None] + xg[None, :]).ravel()      # unit coords of all points
    wq = np.tile(wg, N)
    B, _ = gd1d.basis_eval(N, p, tq)                         # [nq*N, n1]
    uq = np.einsum("rj,qi,abji->abrq", B, B, U)              # [ny, nx, r(y), q(x)]
    xe = prob.x0 + np.arange(prob.nx) * prob.Hx
    ye = prob.y0 + np.arange(prob.ny) * prob.Hy
    xq = xe[None, :, None, None] + tq[None, None, None, :] * prob.hx
    yq = ye[:, None, None, None] + tq[None, None, :, None] * prob.hy
    err = uq - exact(xq, yq)
    w2 = np.outer(wq, wq) * prob.hx * prob.hy
    return float(np.sqrt(np.sum(err ** 2 * w2[None, None])))
