"""Energy-DG with a GD basis on mapped elements with a variable c^2 -- FP64 oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain quadrature assembly of
dense element matrices and dense direct (Cholesky) element solves.

Paper passages followed:
  * Sec. 2.2, eqs. DG1, DG2, DG1_extra -- the variational statement, now with c^2(x, y)
    inside the integrals;
  * Sec. 2.2.1 -- the fluxes;
  * Sec. 7 and Sec. 7.1 -- the stiffness S_{c^2} = int c^2 grad phi . grad phi is no longer a
    Kronecker sum; the paper names the mapped (non-Cartesian) element as the other
    case where this happens.

Readings (the paper gives no formulas for mapped elements):
  * Isoparametric GD elements: each element is the image of the reference square
    (r, s) in [0, 1]^2 (GD grid spacing 1/N) under the map (X, Y)(r, s) interpolated
    in the same GD basis from nodal coordinates; c^2 is interpolated the same way from
    nodal samples.  Because phi_i(0) = delta_i0 and phi_i(1) = delta_iN, a face sees only
    its own nodes, so two neighbours agree on the face geometry and on c^2 there.
  * Volume integrals use (p+1) x (p+1) Gauss-Legendre points per cell, face integrals
    (p+1) points per face cell; with A = d(X,Y)/d(r,s), J = det A,
    K = c^2 J A^{-1} A^{-T}:  M_J = int phi phi J, S_K = int grad_r phi^T K grad_r phi,
    w = int phi J.
  * On a face with reference outward normal Nh, c^2 (n . grad phi) dS = (Nh^T K grad_r phi) ds
    and dS = s_J ds, s_J = |dX/d(tangent)|; the outward normal derivative is
    a = Nh^T K grad_r u / (c^2 s_J).
  * The extra equation enters as S_hat = S_K + (kappa/|Omega_k|) w w^T with
    kappa = int c^2 J / int J (the element-mean c^2); y = S_hat^{-1} F_u does not depend on it.
  * xi of the upwind flux is a fixed reference speed (xi = 1 by default).

Array layout as in ``dg2d``: [ny, nx, N+1 (iy), N+1 (ix)]; X, Y, c2 are nodal arrays of
the same shape.
"""
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import gd1d
from .dg2d import face_alpha, flux_params, face_sigmas


@dataclass
class GenProblem:
    nx: int
    ny: int
    N: int
    p: int
    flux: str = "upwind"
    xi: float = 1.0
    # boundary kind of the E, W, N, S sides of the element grid (as in dg2d.CartProblem):
    # a wall face takes the mirror exterior state of the element's own traces at its face
    # points (Dirichlet: a_ext = -a, v_ext = -v; Neumann: a_ext = a, v_ext = v)
    bc: tuple = ("periodic", "periodic", "periodic", "periodic")
    # source terms (g_nodal [ny, nx, N+1, N+1] at the physical nodes, omega, phase):
    # f = sum_k sin(omega_k t + phase_k) g_k with g_k represented by its GD interpolant,
    # so the load vector of DG2 is M_J g_k and dV/dt gains sum_k s_k(t) g_k
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


FACES = ("E", "W", "N", "S")


class GenOps:
    """Assembled element data of a mapped, variable-coefficient element grid."""

    def __init__(self, prob: GenProblem, X, Y, c2):
        gd1d.check_degree(prob.N, prob.p)
        self.prob = prob
        N, p = prob.N, prob.p
        self.n1 = n1 = N + 1
        self.X, self.Y, self.c2 = (np.asarray(a, dtype=np.float64) for a in (X, Y, c2))
        ne = prob.nx * prob.ny
        shp = (prob.ny, prob.nx, n1, n1)
        assert self.X.shape == shp and self.Y.shape == shp and self.c2.shape == shp
        Xe = self.X.reshape(ne, n1, n1)
        Ye = self.Y.reshape(ne, n1, n1)
        Ce = self.c2.reshape(ne, n1, n1)
        xg, wg = gd1d.gauss_legendre(p + 1)
        M = np.zeros((ne, n1 * n1, n1 * n1))
        S = np.zeros((ne, n1 * n1, n1 * n1))
        w = np.zeros((ne, n1 * n1))
        kint = np.zeros((ne, 3))            # int K_rr, int K_ss, int c^2 J
        # ---- volume: loop over cells, vectorised over elements --------------------
        # On cell (kx, ky) only the (p+1)^2 functions of the two stencil windows are
        # non-zero; local matrices are formed on those and added into the element ones.
        m = p + 1
        wq = np.outer(wg, wg) / (N * N)                          # [qb, qa]
        for kx in range(N):
            sx = gd1d.window_start(kx, N, p)
            Bx, Dx = gd1d.basis_on_cell(kx, N, p, kx + xg)       # [q, n1] (t-derivs)
            Bx, Dx = Bx[:, sx:sx + m], Dx[:, sx:sx + m] * N      # d/dr on the window
            for ky in range(N):
                sy = gd1d.window_start(ky, N, p)
                By, Dy = gd1d.basis_on_cell(ky, N, p, ky + xg)
                By, Dy = By[:, sy:sy + m], Dy[:, sy:sy + m] * N
                # phi_{jy,jx}(qb, qa) and reference gradients: [qb, qa, jy, jx]
                phi = np.einsum("bj,ai->baji", By, Bx)
                dr = np.einsum("bj,ai->baji", By, Dx)
                ds = np.einsum("bj,ai->baji", Dy, Bx)
                Xl = Xe[:, sy:sy + m, sx:sx + m]
                Yl = Ye[:, sy:sy + m, sx:sx + m]
                Cl = Ce[:, sy:sy + m, sx:sx + m]
                Xr = np.einsum("baji,eji->eba", dr, Xl)
                Xs = np.einsum("baji,eji->eba", ds, Xl)
                Yr = np.einsum("baji,eji->eba", dr, Yl)
                Ys = np.einsum("baji,eji->eba", ds, Yl)
                cq = np.einsum("baji,eji->eba", phi, Cl)
                J = Xr * Ys - Xs * Yr
                # K = c^2 J A^{-1} A^{-T}, A = [[Xr, Xs], [Yr, Ys]]
                Krr = cq * (Xs * Xs + Ys * Ys) / J
                Kss = cq * (Xr * Xr + Yr * Yr) / J
                Krs = -cq * (Xr * Xs + Yr * Ys) / J
                P = phi.reshape(m, m, m * m)
                R = dr.reshape(m, m, m * m)
                Sd = ds.reshape(m, m, m * m)
                Mloc = np.einsum("ba,eba,bai,baj->eij", wq, J, P, P, optimize=True)
                Sloc = (np.einsum("ba,eba,bai,baj->eij", wq, Krr, R, R, optimize=True)
                        + np.einsum("ba,eba,bai,baj->eij", wq, Kss, Sd, Sd, optimize=True)
                        + np.einsum("ba,eba,bai,baj->eij", wq, Krs, R, Sd, optimize=True)
                        + np.einsum("ba,eba,bai,baj->eij", wq, Krs, Sd, R, optimize=True))
                gidx = ((sy + np.arange(m))[:, None] * n1 + (sx + np.arange(m))[None, :]).ravel()
                M[:, gidx[:, None], gidx[None, :]] += Mloc
                S[:, gidx[:, None], gidx[None, :]] += Sloc
                w[:, gidx] += np.einsum("ba,eba,bai->ei", wq, J, P)
                kint[:, 0] += np.einsum("ba,eba->e", wq, Krr)
                kint[:, 1] += np.einsum("ba,eba->e", wq, Kss)
                kint[:, 2] += np.einsum("ba,eba->e", wq, cq * J)
        self.M, self.S, self.w = M, S, w
        self.area = w.sum(axis=1)
        self.kappa = kint[:, 2] / self.area
        self.kbar_rr, self.kbar_ss = kint[:, 0], kint[:, 1]
        self.Shat = S + (self.kappa / self.area)[:, None, None] * np.einsum("ei,ej->eij", w, w)
        self._cS = [sla.cho_factor(A) for A in self.Shat]
        self._cM = [sla.cho_factor(A) for A in M]
        # ---- faces --------------------------------------------------------------
        self.faces = {f: self._face(f, Xe, Ye, Ce, xg, wg) for f in FACES}

    def _face(self, f, Xe, Ye, Ce, xg, wg):
        """Quadrature data of one face of every element.

        Returns a dict with the along-face basis B, D [q, n1], the normal-direction
        derivative vector dn [n1] (d/dr or d/ds of the basis at the face), the index of
        the face node row/column, Kn = K Nh at the points [e, q, 2], c2sJ = c^2 s_J [e, q],
        and the weights wq [q].
        """
        N, p, n1 = self.prob.N, self.prob.p, self.n1
        tq = (np.arange(N)[:, None] + xg[None, :]).ravel()
        wq = np.tile(wg, N) / N
        Bt, Dt = gd1d.basis_eval(N, p, tq)
        Dt = Dt * N
        dLh, dRh = gd1d.face_vectors_unit(N, p)
        if f in ("E", "W"):
            node = N if f == "E" else 0
            dn = (dRh if f == "E" else dLh) * N
            Nh = np.array([1.0, 0.0]) if f == "E" else np.array([-1.0, 0.0])
            # along-face coordinate s (index iy); normal coordinate r (index ix)
            Xr = np.einsum("i,qj,eji->eq", dn, Bt, Xe)
            Yr = np.einsum("i,qj,eji->eq", dn, Bt, Ye)
            Xs = np.einsum("qj,ej->eq", Dt, Xe[:, :, node])
            Ys = np.einsum("qj,ej->eq", Dt, Ye[:, :, node])
            cq = np.einsum("qj,ej->eq", Bt, Ce[:, :, node])
            sJ = np.sqrt(Xs * Xs + Ys * Ys)
        else:
            node = N if f == "N" else 0
            dn = (dRh if f == "N" else dLh) * N
            Nh = np.array([0.0, 1.0]) if f == "N" else np.array([0.0, -1.0])
            # along-face coordinate r (index ix); normal coordinate s (index iy)
            Xs = np.einsum("j,qi,eji->eq", dn, Bt, Xe)
            Ys = np.einsum("j,qi,eji->eq", dn, Bt, Ye)
            Xr = np.einsum("qi,ei->eq", Dt, Xe[:, node, :])
            Yr = np.einsum("qi,ei->eq", Dt, Ye[:, node, :])
            cq = np.einsum("qi,ei->eq", Bt, Ce[:, node, :])
            sJ = np.sqrt(Xr * Xr + Yr * Yr)
        J = Xr * Ys - Xs * Yr
        Krr = cq * (Xs * Xs + Ys * Ys) / J
        Kss = cq * (Xr * Xr + Yr * Yr) / J
        Krs = -cq * (Xr * Xs + Yr * Ys) / J
        Kn = np.stack([Krr * Nh[0] + Krs * Nh[1], Krs * Nh[0] + Kss * Nh[1]], axis=-1)
        return dict(B=Bt, D=Dt, dn=dn, node=node, Kn=Kn, c2sJ=cq * sJ, wq=wq)

    # ---- per-element operators --------------------------------------------------------
    def apply_S(self, U):
        ny, nx, n1, _ = U.shape
        return np.einsum("eij,ej->ei", self.S, U.reshape(ny * nx, -1)).reshape(U.shape)

    def solve_Shat(self, F):
        ny, nx, n1, _ = F.shape
        b = F.reshape(ny * nx, -1)
        return np.stack([sla.cho_solve(c, bb) for c, bb in zip(self._cS, b)]).reshape(F.shape)

    def solve_M(self, F):
        ny, nx, n1, _ = F.shape
        b = F.reshape(ny * nx, -1)
        return np.stack([sla.cho_solve(c, bb) for c, bb in zip(self._cM, b)]).reshape(F.shape)


def _grad_u_face(fd, f, Ue):
    """Reference gradient (d/dr, d/ds) of u at the face points: [e, q, 2]."""
    B, D, dn, node = fd["B"], fd["D"], fd["dn"], fd["node"]
    if f in ("E", "W"):
        ur = np.einsum("i,qj,eji->eq", dn, B, Ue)
        us = np.einsum("qj,ej->eq", D, Ue[:, :, node])
    else:
        us = np.einsum("j,qi,eji->eq", dn, B, Ue)
        ur = np.einsum("qi,ei->eq", D, Ue[:, node, :])
    return np.stack([ur, us], axis=-1)


def _value_face(fd, f, Ve):
    B, node = fd["B"], fd["node"]
    if f in ("E", "W"):
        return np.einsum("qj,ej->eq", B, Ve[:, :, node])
    return np.einsum("qi,ei->eq", B, Ve[:, node, :])


def face_traces(U, V, ops):
    """Outward normal derivative a and value v of (u, v) at the face points, per face."""
    prob = ops.prob
    ne, n1 = prob.nx * prob.ny, ops.n1
    Ue, Ve = U.reshape(ne, n1, n1), V.reshape(ne, n1, n1)
    out = {}
    for f in FACES:
        fd = ops.faces[f]
        g = _grad_u_face(fd, f, Ue)
        a = np.einsum("eqk,eqk->eq", fd["Kn"], g) / fd["c2sJ"]
        out[f] = (a, _value_face(fd, f, Ve))
    return out


def _neighbour(arr, f, prob):
    """Values of the periodic neighbour across face f (its opposite face), [e, q]."""
    a = arr.reshape(prob.ny, prob.nx, -1)
    if f == "E":
        a = np.roll(a, -1, axis=1)
    elif f == "W":
        a = np.roll(a, +1, axis=1)
    elif f == "N":
        a = np.roll(a, -1, axis=0)
    else:
        a = np.roll(a, +1, axis=0)
    return a.reshape(prob.ny * prob.nx, -1)


OPP = {"E": "W", "W": "E", "N": "S", "S": "N"}


def _exterior(tr, f, prob):
    """Exterior state (a_nb, v_nb) at the points of face f of every element: the periodic
    neighbour's traces on its opposite face, or on a wall face the mirror of the element's
    own traces."""
    an = _neighbour(tr[OPP[f]][0], f, prob)
    vn = _neighbour(tr[OPP[f]][1], f, prob)
    kind = prob.bc["EWNS".index(f)]
    if kind != "periodic":
        sgn = -1.0 if kind == "dirichlet" else 1.0
        side = {"E": (slice(None), -1), "W": (slice(None), 0), "N": (-1, slice(None)),
                "S": (0, slice(None))}[f]
        wall = np.zeros((prob.ny, prob.nx), dtype=bool)
        wall[side] = True
        wall = wall.ravel()
        an[wall] = sgn * tr[f][0][wall]
        vn[wall] = sgn * tr[f][1][wall]
    return an, vn


def _face_alphas(prob, f):
    """alpha of face f (dg2d.face_alpha) for every element, flat [e] (wall faces differ)."""
    al = np.full((prob.ny, prob.nx), face_alpha(prob.flux, f))
    if prob.bc["EWNS".index(f)] != "periodic":
        side = {"E": (slice(None), -1), "W": (slice(None), 0), "N": (-1, slice(None)),
                "S": (0, slice(None))}[f]
        al[side] = face_alpha(prob.flux, f, wall=True)
    return al.ravel()


def lifts(U, V, ops):
    """F_u,i = int c^2 (n . grad phi_i)(v* - v) dS and F_v,i = int c^2 phi_i n.(grad u)* dS."""
    prob = ops.prob
    _, beta, tau = flux_params(prob.flux, prob.xi)
    ne, n1 = prob.nx * prob.ny, ops.n1
    tr = face_traces(U, V, ops)
    Fu = np.zeros((ne, n1, n1))
    Fv = np.zeros((ne, n1, n1))
    for f in FACES:
        fd = ops.faces[f]
        a, v = tr[f]
        an, vn = _exterior(tr, f, prob)
        su, sv = face_sigmas(a, v, an, vn, _face_alphas(prob, f)[:, None], beta, tau)
        wsu = fd["wq"][None, :] * su
        wsv = fd["wq"][None, :] * sv * fd["c2sJ"]
        B, D, dn, node = fd["B"], fd["D"], fd["dn"], fd["node"]
        Knr, Kns = fd["Kn"][..., 0], fd["Kn"][..., 1]
        if f in ("E", "W"):
            # Nh^T K grad_r phi_{iy,ix} = Knr dn[ix] B[q,iy] + Kns delta_{ix,node} D[q,iy]
            Fu += np.einsum("eq,i,qj->eji", wsu * Knr, dn, B)
            Fu[:, :, node] += np.einsum("eq,qj->ej", wsu * Kns, D)
            Fv[:, :, node] += np.einsum("eq,qj->ej", wsv, B)
        else:
            Fu += np.einsum("eq,j,qi->eji", wsu * Kns, dn, B)
            Fu[:, node, :] += np.einsum("eq,qi->ei", wsu * Knr, D)
            Fv[:, node, :] += np.einsum("eq,qi->ei", wsv, B)
    shp = (prob.ny, prob.nx, n1, n1)
    return Fu.reshape(shp), Fv.reshape(shp)


def rhs(U, V, ops, t=0.0):
    """S_hat (dU/dt - V) = F_u,   M_J dV/dt = -S_K U + F_v + sum_k s_k(t) M_J g_k
    (dense direct solves; the source term's solve is exact: M_J^-1 M_J g_k = g_k)."""
    Fu, Fv = lifts(U, V, ops)
    return V + ops.solve_Shat(Fu), ops.solve_M(-ops.apply_S(U) + Fv) + forcing_term(ops.prob, t)


def forcing_term(prob, t):
    """sum_k sin(omega_k t + phase_k) g_k (nodal; zero without source terms)."""
    out = 0.0
    for g, omega, phase in prob.forcing:
        out = out + np.sin(omega * t + phase) * np.asarray(g, dtype=np.float64)
    return out


def rk4_step(U, V, dt, f):
    k1u, k1v = f(U, V)
    k2u, k2v = f(U + 0.5 * dt * k1u, V + 0.5 * dt * k1v)
    k3u, k3v = f(U + 0.5 * dt * k2u, V + 0.5 * dt * k2v)
    k4u, k4v = f(U + dt * k3u, V + dt * k3v)
    return (U + dt / 6.0 * (k1u + 2 * k2u + 2 * k3u + k4u),
            V + dt / 6.0 * (k1v + 2 * k2v + 2 * k3v + k4v))


def run(U, V, ops, dt, steps, f=None, t0=0.0):
    """steps RK4 steps from time t0; a source term makes the stages time-dependent
    (stage times t, t + dt/2, t + dt/2, t + dt).  f: a custom right-hand side (U, V)."""
    if f is not None or not ops.prob.forcing:
        f = f or (lambda a, b: rhs(a, b, ops))
        for _ in range(steps):
            U, V = rk4_step(U, V, dt, f)
        return U, V
    for s in range(steps):
        t = t0 + s * dt
        k1u, k1v = rhs(U, V, ops, t)
        k2u, k2v = rhs(U + 0.5 * dt * k1u, V + 0.5 * dt * k1v, ops, t + 0.5 * dt)
        k3u, k3v = rhs(U + 0.5 * dt * k2u, V + 0.5 * dt * k2v, ops, t + 0.5 * dt)
        k4u, k4v = rhs(U + dt * k3u, V + dt * k3v, ops, t + dt)
        U = U + dt / 6.0 * (k1u + 2 * k2u + 2 * k3u + k4u)
        V = V + dt / 6.0 * (k1v + 2 * k2v + 2 * k3v + k4v)
    return U, V


def energy(U, V, ops):
    """sum_k 1/2 V^T M_J V + 1/2 U^T S_K U."""
    ne = ops.prob.nx * ops.prob.ny
    u, v = U.reshape(ne, -1), V.reshape(ne, -1)
    return 0.5 * float(np.einsum("ei,eij,ej->", v, ops.M, v) + np.einsum("ei,eij,ej->", u, ops.S, u))


def energy_rate(U, V, ops):
    Fu, Fv = lifts(U, V, ops)
    return float(np.sum(U * Fu) + np.sum(V * Fv))


def face_dissipation(U, V, ops):
    """-sum over faces of int c^2 (beta (a + a_nb)^2 + tau (v_nb - v)^2) dS: every face of
    every element with weight 1/2, so an interior face (seen from both sides) counts once
    and a wall face (seen from its element only, against the mirror state) counts half --
    the share of the doubled domain that the wall's half owns."""
    prob = ops.prob
    _, beta, tau = flux_params(prob.flux, prob.xi)
    tr = face_traces(U, V, ops)
    tot = 0.0
    for f in FACES:
        fd = ops.faces[f]
        a, v = tr[f]
        an, vn = _exterior(tr, f, prob)
        integrand = fd["c2sJ"] * (beta * (a + an) ** 2 + tau * (vn - v) ** 2)
        tot -= 0.5 * float(np.sum(fd["wq"][None, :] * integrand))
    return tot
