"""Energy-DG with a GD basis on a Cartesian grid of box elements in three dimensions,
constant c -- oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain FP64, nodal state, dense
direct element solves.

The paper states the method for d = 2 and d = 3 alike; the passages followed:
  * Sec. 2.2: elements are boxes prod_l [L_l, R_l], l in {x, y, z}, carrying the tensor
    product of the 1D GD space (same degree and N in every direction); the element-wise
    statements DG1, DG2 and DG1_extra.
  * Sec. 2.2.1: the fluxes v*, (grad u)* with (alpha, beta, tau) -- central, upwind and
    (with the orientation reading of dg2d.face_alpha: v* from the element on the
    low-coordinate side, alpha = 1/2 on walls) alternating.
  * Sec. 3.1 / Sec. 3.2: the Kronecker forms, in 3D
      M = M_x (x) M_y (x) M_z,   S = S_x (x) M_y (x) M_z + M_x (x) S_y (x) M_z
                                      + M_x (x) M_y (x) S_z,
    with the rank-one surface terms on each of the six faces.
  * Sec. 3.3 / Sec. 6: classical RK4.
Readings as in dg2d (the tau term, the variational rather than the matrix form, the
extra equation as S_hat = c^2 S + (kappa/|Omega_k|) w w^T with kappa = c^2, nodal
interpolation of the data, walls as mirror states).

Array layout: a field is [nz, ny, nx, N+1 (iz), N+1 (iy), N+1 (ix)]; element (ex, ey, ez)
covers [x0 + ex Hx, x0 + (ex+1) Hx] x [y0 + ey Hy, ...] x [z0 + ez Hz, ...]; node
(ix, iy, iz) sits at (x0 + ex Hx + ix hx, ...); nodes on faces are duplicated per element.
Faces: E / W (x = R / L), N / S (y = R / L), T / B (z = R / L).
"""
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import gd1d
from .dg2d import face_alpha, face_sigmas, flux_params

FACES = ("E", "W", "N", "S", "T", "B")
OPP = {"E": "W", "W": "E", "N": "S", "S": "N", "T": "B", "B": "T"}
# element-grid axis (of [nz, ny, nx]) and roll shift that bring the neighbour across f
_NB = {"E": (2, -1), "W": (2, +1), "N": (1, -1), "S": (1, +1), "T": (0, -1), "B": (0, +1)}
# the elements touching each side of the box
_SIDE = {"E": (slice(None), slice(None), -1), "W": (slice(None), slice(None), 0),
         "N": (slice(None), -1, slice(None)), "S": (slice(None), 0, slice(None)),
         "T": (-1, slice(None), slice(None)), "B": (0, slice(None), slice(None))}


@dataclass
class CartProblem3:
    nx: int
    ny: int
    nz: int
    N: int
    p: int
    Lx: float = 1.0
    Ly: float = 1.0
    Lz: float = 1.0
    x0: float = 0.0
    y0: float = 0.0
    z0: float = 0.0
    c2: float = 1.0
    flux: str = "central"
    xi: float = 1.0
    # boundary kind of the E, W, N, S, T, B sides: "periodic", "dirichlet" or "neumann"
    bc: tuple = ("periodic",) * 6

    def __post_init__(self):
        kinds = ("periodic", "dirichlet", "neumann")
        bc = tuple(self.bc)
        if len(bc) != 6 or any(k not in kinds for k in bc):
            raise ValueError("bc: six of %s (E, W, N, S, T, B)" % (kinds,))
        for a, b in ((0, 1), (2, 3), (4, 5)):
            if (bc[a] == "periodic") != (bc[b] == "periodic"):
                raise ValueError("a direction is periodic on both sides or on neither")
        self.bc = bc

    @property
    def H(self):
        return self.Lx / self.nx, self.Ly / self.ny, self.Lz / self.nz

    @property
    def h(self):
        return tuple(Hd / self.N for Hd in self.H)


class CartOps3:
    """1D and 3D element operators of one box element (Sec. 3.1, Sec. 3.2)."""

    def __init__(self, prob: CartProblem3):
        gd1d.check_degree(prob.N, prob.p)
        self.prob = prob
        self.n1 = n1 = prob.N + 1
        Hx, Hy, Hz = prob.H
        self.Mx, self.Sx, self.dLx, self.dRx = gd1d.element_1d(prob.N, prob.p, Hx)
        self.My, self.Sy, self.dLy, self.dRy = gd1d.element_1d(prob.N, prob.p, Hy)
        self.Mz, self.Sz, self.dLz, self.dRz = gd1d.element_1d(prob.N, prob.p, Hz)
        # flattened index (iz * n1 + iy) * n1 + ix: an operator A_z on z, B_y on y and C_x
        # on x is kron(A_z, kron(B_y, C_x))
        k3 = lambda a, b, c: np.kron(a, np.kron(b, c))
        self.M3 = k3(self.Mz, self.My, self.Mx)
        self.S3 = (k3(self.Mz, self.My, self.Sx) + k3(self.Mz, self.Sy, self.Mx)
                   + k3(self.Sz, self.My, self.Mx))
        one = np.ones(n1)
        self.w = k3(self.Mz @ one, self.My @ one, self.Mx @ one)
        vol = Hx * Hy * Hz
        self.kappa = prob.c2
        self.Shat = prob.c2 * self.S3 + (self.kappa / vol) * np.outer(self.w, self.w)
        self._chol_S = sla.cho_factor(self.Shat)
        self._chol_M = sla.cho_factor(self.M3)

    def _solve(self, chol, F):
        n = F.shape[0] * F.shape[1] * F.shape[2]
        return sla.cho_solve(chol, F.reshape(n, -1).T).T.reshape(F.shape)

    def solve_Shat(self, F):
        return self._solve(self._chol_S, F)

    def solve_M(self, F):
        return self._solve(self._chol_M, F)


def traces(U, V, ops):
    """Outward normal derivative a_f and value v_f on the six faces: dict f -> (a, v),
    each [nz, ny, nx, n1, n1] indexed by the two face coordinates in the field's order
    (E/W: [iz, iy]; N/S: [iz, ix]; T/B: [iy, ix])."""
    return {
        "E": (np.einsum("i,...zyi->...zy", ops.dRx, U), V[..., :, :, -1]),
        "W": (-np.einsum("i,...zyi->...zy", ops.dLx, U), V[..., :, :, 0]),
        "N": (np.einsum("j,...zjx->...zx", ops.dRy, U), V[..., :, -1, :]),
        "S": (-np.einsum("j,...zjx->...zx", ops.dLy, U), V[..., :, 0, :]),
        "T": (np.einsum("k,...kyx->...yx", ops.dRz, U), V[..., -1, :, :]),
        "B": (-np.einsum("k,...kyx->...yx", ops.dLz, U), V[..., 0, :, :]),
    }


def neighbour_traces(tr, bc):
    """Traces of the neighbour across each face (its opposite face), or on a wall face
    the mirror of the element's own (Dirichlet: -a, -v; Neumann: a, v)."""
    nb = {}
    for f in FACES:
        ax, sh = _NB[f]
        nb[f] = tuple(np.roll(t, sh, axis=ax) for t in tr[OPP[f]])
    for f, kind in zip(FACES, bc):
        if kind == "periodic":
            continue
        sgn = -1.0 if kind == "dirichlet" else 1.0
        for k in (0, 1):
            nb[f][k][_SIDE[f]] = sgn * tr[f][k][_SIDE[f]]
    return nb


def face_alphas(prob, f):
    """alpha of face f for every element, [nz, ny, nx] (T like N, B like S; walls 1/2)."""
    f2 = {"T": "N", "B": "S"}.get(f, f)
    al = np.full((prob.nz, prob.ny, prob.nx), face_alpha(prob.flux, f2))
    if prob.bc[FACES.index(f)] != "periodic":
        al[_SIDE[f]] = face_alpha(prob.flux, f2, wall=True)
    return al


def lifts(U, V, ops):
    """Face terms F_u, F_v of DG1 / DG2 for every element.

    F_u,i = int_{dOmega} c^2 (n . grad phi_i)(v* - v) and F_v,i = int c^2 phi_i n.(grad u)*.
    On a face the traces are GD functions of the two face coordinates, so the face
    integrals are products with the two 1D mass matrices along the face.
    """
    prob = ops.prob
    _, beta, tau = flux_params(prob.flux, prob.xi)
    c2 = prob.c2
    tr = traces(U, V, ops)
    nb = neighbour_traces(tr, prob.bc)
    Fu = np.zeros_like(U)
    Fv = np.zeros_like(V)
    Mx, My, Mz = ops.Mx, ops.My, ops.Mz
    for f in FACES:
        su, sv = face_sigmas(tr[f][0], tr[f][1], nb[f][0], nb[f][1],
                             face_alphas(prob, f)[..., None, None], beta, tau)
        if f in ("E", "W"):          # face arrays [iz, iy]
            mu = np.einsum("ac,bd,...cd->...ab", Mz, My, su, optimize=True)
            mv = np.einsum("ac,bd,...cd->...ab", Mz, My, sv, optimize=True)
            d = ops.dRx if f == "E" else -ops.dLx
            Fu += c2 * np.einsum("i,...zy->...zyi", d, mu)
            Fv[..., :, :, -1 if f == "E" else 0] += c2 * mv
        elif f in ("N", "S"):        # face arrays [iz, ix]
            mu = np.einsum("ac,bd,...cd->...ab", Mz, Mx, su, optimize=True)
            mv = np.einsum("ac,bd,...cd->...ab", Mz, Mx, sv, optimize=True)
            d = ops.dRy if f == "N" else -ops.dLy
            Fu += c2 * np.einsum("j,...zx->...zjx", d, mu)
            Fv[..., :, -1 if f == "N" else 0, :] += c2 * mv
        else:                        # face arrays [iy, ix]
            mu = np.einsum("ac,bd,...cd->...ab", My, Mx, su, optimize=True)
            mv = np.einsum("ac,bd,...cd->...ab", My, Mx, sv, optimize=True)
            d = ops.dRz if f == "T" else -ops.dLz
            Fu += c2 * np.einsum("k,...yx->...kyx", d, mu)
            Fv[..., -1 if f == "T" else 0, :, :] += c2 * mv
    return Fu, Fv


def apply_S3(U, ops):
    """(S_x (x) M_y (x) M_z + M_x (x) S_y (x) M_z + M_x (x) M_y (x) S_z) U per element."""
    e = "ka,jb,ic,...abc->...kji"
    return (np.einsum(e, ops.Mz, ops.My, ops.Sx, U, optimize=True)
            + np.einsum(e, ops.Mz, ops.Sy, ops.Mx, U, optimize=True)
            + np.einsum(e, ops.Sz, ops.My, ops.Mx, U, optimize=True))


def rhs(U, V, ops):
    """(dU/dt, dV/dt): S_hat (dU/dt - V) = F_u and M dV/dt = -c^2 S U + F_v."""
    Fu, Fv = lifts(U, V, ops)
    y = ops.solve_Shat(Fu)
    z = ops.solve_M(-ops.prob.c2 * apply_S3(U, ops) + Fv)
    return V + y, z


def run(U, V, ops, dt, steps):
    """steps classical RK4 steps."""
    f = lambda a, b: rhs(a, b, ops)
    for _ in range(steps):
        k1u, k1v = f(U, V)
        k2u, k2v = f(U + 0.5 * dt * k1u, V + 0.5 * dt * k1v)
        k3u, k3v = f(U + 0.5 * dt * k2u, V + 0.5 * dt * k2v)
        k4u, k4v = f(U + dt * k3u, V + dt * k3v)
        U = U + dt / 6.0 * (k1u + 2 * k2u + 2 * k3u + k4u)
        V = V + dt / 6.0 * (k1v + 2 * k2v + 2 * k3v + k4v)
    return U, V


def energy(U, V, ops):
    """sum_k 1/2 V^T M V + 1/2 c^2 U^T S U."""
    n1 = ops.n1
    u = U.reshape(-1, n1 ** 3)
    v = V.reshape(-1, n1 ** 3)
    return (0.5 * np.einsum("ei,ij,ej->", v, ops.M3, v)
            + 0.5 * ops.prob.c2 * np.einsum("ei,ij,ej->", u, ops.S3, u))


def energy_rate(U, V, ops):
    """dE/dt = sum_k (U^T F_u + V^T F_v) (from DG1, DG2 with phi_u = U, phi_v = V)."""
    Fu, Fv = lifts(U, V, ops)
    return float(np.sum(U * Fu) + np.sum(V * Fv))


def node_coords(prob):
    """Physical node coordinates X, Y, Z, each [nz, ny, nx, n1, n1, n1]."""
    n1 = prob.N + 1
    Hx, Hy, Hz = prob.H
    hx, hy, hz = prob.h
    i = np.arange(n1)
    shp = (prob.nz, prob.ny, prob.nx, n1, n1, n1)
    X = prob.x0 + np.arange(prob.nx)[None, None, :, None, None, None] * Hx \
        + i[None, None, None, None, None, :] * hx
    Y = prob.y0 + np.arange(prob.ny)[None, :, None, None, None, None] * Hy \
        + i[None, None, None, None, :, None] * hy
    Z = prob.z0 + np.arange(prob.nz)[:, None, None, None, None, None] * Hz \
        + i[None, None, None, :, None, None] * hz
    return (np.broadcast_to(X, shp).copy(), np.broadcast_to(Y, shp).copy(),
            np.broadcast_to(Z, shp).copy())
