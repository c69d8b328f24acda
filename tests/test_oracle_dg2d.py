"""Pins of the 2D constant-coefficient energy-DG oracle (Sec. 2.2, Sec. 3, Sec. 6).

What fixes the answer here: the Kronecker structure of Sec. 3.1, the energy
identity implied by DG1 / DG2 with the fluxes of Sec. 2.2.1, exact conservation of
constants, the Taylor form of classical RK4 on a linear system, exact standing
and travelling wave solutions and the paper's fourth-order 2D rate for p = 3.
"""
import numpy as np
import pytest

from oracle import dg2d, gd1d
from paper_2105_01722_amd import inputs


def _prob(n=2, N=6, p=3, flux="central", c2=1.0, Lx=1.0, Ly=1.0):
    return dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux=flux, c2=c2, Lx=Lx, Ly=Ly,
                            xi=np.sqrt(c2))


def _rand_state(prob, seed):
    rng = np.random.default_rng(seed)
    shp = (prob.ny, prob.nx, prob.N + 1, prob.N + 1)
    return rng.standard_normal(shp), rng.standard_normal(shp)


def _dense_L(ops, prob):
    n1 = prob.N + 1
    sz = prob.nx * prob.ny * n1 * n1
    L = np.zeros((2 * sz, 2 * sz))
    shp = (prob.ny, prob.nx, n1, n1)
    for k in range(2 * sz):
        z = np.zeros(2 * sz)
        z[k] = 1.0
        a, b = dg2d.rhs(z[:sz].reshape(shp), z[sz:].reshape(shp), ops)
        L[:, k] = np.concatenate([a.ravel(), b.ravel()])
    return L


def test_kronecker_structure_matches_2d_quadrature():
    """Sec. 3.1: the element mass is M_x (x) M_y and the stiffness S_x (x) M_y + M_x (x) S_y.
    Checked against direct 2D Gauss integration of the tensor-product basis."""
    prob = _prob(n=1, N=5, p=3, Lx=0.7, Ly=1.3)
    ops = dg2d.CartOps(prob)
    N, p = prob.N, prob.p
    xg, wg = gd1d.gauss_legendre(p + 1)
    n1 = N + 1
    M = np.zeros((n1 * n1, n1 * n1))
    S = np.zeros_like(M)
    for kx in range(N):
        for ky in range(N):
            bx, dbx = gd1d.basis_on_cell(kx, N, p, kx + xg)
            by, dby = gd1d.basis_on_cell(ky, N, p, ky + xg)
            for a in range(p + 1):
                for b in range(p + 1):
                    w = wg[a] * wg[b] * prob.hx * prob.hy
                    phi = np.outer(by[b], bx[a]).ravel()          # index iy*n1 + ix
                    gx = np.outer(by[b], dbx[a]).ravel() / prob.hx
                    gy = np.outer(dby[b], bx[a]).ravel() / prob.hy
                    M += w * np.outer(phi, phi)
                    S += w * (np.outer(gx, gx) + np.outer(gy, gy))
    np.testing.assert_allclose(ops.M2, M, atol=1e-15)
    np.testing.assert_allclose(ops.S2, S, atol=1e-12)


@pytest.mark.parametrize("N,p", [(6, 3), (5, 5), (8, 7)])
def test_energy_conserved_central(N, p):
    """Sec. 2.2.1: the central flux (beta = tau = 0) is energy conserving.  With
    (dU, dV) from the full right-hand side (solves included),
    d/dt [1/2 V^T M V + 1/2 c^2 U^T S U] = V^T M dV + c^2 U^T S dU = 0."""
    prob = _prob(n=3, N=N, p=p, flux="central", c2=1.7)
    ops = dg2d.CartOps(prob)
    U, V = _rand_state(prob, 1)
    dU, dV = dg2d.rhs(U, V, ops)
    n = prob.nx * prob.ny
    u, v = U.reshape(n, -1), V.reshape(n, -1)
    du, dv = dU.reshape(n, -1), dV.reshape(n, -1)
    rate = np.einsum("ei,ij,ej->", v, ops.M2, dv) + prob.c2 * np.einsum("ei,ij,ej->", u, ops.S2, du)
    scale = np.abs(np.einsum("ei,ij,ej->e", v, ops.M2, dv)).sum()
    assert abs(rate) < 1e-12 * scale
    assert abs(dg2d.energy_rate(U, V, ops)) < 1e-12 * scale


@pytest.mark.parametrize("N,p", [(6, 3), (5, 5)])
def test_energy_dissipation_upwind(N, p):
    """Sec. 2.2.1 upwind flux: summing DG1 / DG2 over elements with the test functions
    U, V leaves only face terms; per face they add to
    -c^2 int (beta (a + a_nb)^2 + tau (v_nb - v)^2), a, a_nb the outward normal
    derivatives and v, v_nb the values on the two sides."""
    c2 = 2.3
    prob = _prob(n=3, N=N, p=p, flux="upwind", c2=c2)
    ops = dg2d.CartOps(prob)
    U, V = _rand_state(prob, 2)
    dU, dV = dg2d.rhs(U, V, ops)
    n = prob.nx * prob.ny
    rate = (np.einsum("ei,ij,ej->", V.reshape(n, -1), ops.M2, dV.reshape(n, -1))
            + c2 * np.einsum("ei,ij,ej->", U.reshape(n, -1), ops.S2, dU.reshape(n, -1)))
    beta, tau = 0.5 * np.sqrt(c2), 0.5 / np.sqrt(c2)
    # traces computed here directly from the nodal data (one-sided derivatives)
    _, _, dL, dR = gd1d.element_1d(N, p, prob.Hx)
    My = gd1d.element_1d(N, p, prob.Hy)[0]
    expect = 0.0
    for ey in range(prob.ny):
        for ex in range(prob.nx):
            e2 = (ex + 1) % prob.nx                       # east neighbour: x faces
            a1 = U[ey, ex] @ dR                           # d/dx at x = R, along y
            a2 = -(U[ey, e2] @ dL)                        # outward (-x) derivative of neighbour
            jv = V[ey, e2][:, 0] - V[ey, ex][:, -1]
            expect -= c2 * (beta * (a1 + a2) @ My @ (a1 + a2) + tau * jv @ My @ jv)
            n2 = (ey + 1) % prob.ny                       # north neighbour: y faces
            b1 = dR @ U[ey, ex]
            b2 = -(dL @ U[n2, ex])
            jv = V[n2, ex][0, :] - V[ey, ex][-1, :]
            expect -= c2 * (beta * (b1 + b2) @ My @ (b1 + b2) + tau * jv @ My @ jv)
    assert expect < 0
    assert abs(rate - expect) < 1e-11 * abs(expect)


@pytest.mark.parametrize("flux", ["central", "upwind"])
def test_constants_are_steady_and_translate(flux):
    """A constant u with v = 0 is a steady state; a constant v gives dU/dt = v, dV/dt = 0
    (DG1_extra fixes the mean of dU/dt, every face term vanishes on constants)."""
    prob = _prob(n=2, N=7, p=5, flux=flux)
    ops = dg2d.CartOps(prob)
    shp = (2, 2, 8, 8)
    dU, dV = dg2d.rhs(np.full(shp, 3.0), np.zeros(shp), ops)
    assert np.abs(dU).max() < 1e-11 and np.abs(dV).max() < 1e-10
    dU, dV = dg2d.rhs(np.zeros(shp), np.full(shp, -2.0), ops)
    assert np.abs(dU + 2.0).max() < 1e-11 and np.abs(dV).max() < 1e-10


def test_extra_equation_kappa_independent():
    """DG1_extra: S_hat y = F_u with S_hat = c^2 S + (kappa/|Omega|) w w^T has w^T y = 0 and
    the same y for every kappa > 0 (1^T F_u = 0 because the basis sums to one)."""
    prob = _prob(n=2, N=6, p=3, flux="upwind")
    ops = dg2d.CartOps(prob)
    U, V = _rand_state(prob, 3)
    Fu, _ = dg2d.lifts(U, V, ops)
    assert np.abs(Fu.sum(axis=(2, 3))).max() < 1e-11
    y = ops.solve_Shat(Fu)
    assert np.abs(np.einsum("i,abi->ab", ops.w, y.reshape(2, 2, -1))).max() < 1e-12
    area = prob.Hx * prob.Hy
    S2 = ops.Shat + (7.5 / area) * np.outer(ops.w, ops.w)
    y2 = np.linalg.solve(S2, Fu.reshape(4, -1).T).T.reshape(Fu.shape)
    np.testing.assert_allclose(y2, y, atol=1e-11)


def test_rk4_equals_taylor_polynomial():
    """Sec. 3.3 / Sec. 6: classical RK4 on the linear system Z' = L Z is Z <- R4(dt L) Z with
    R4(z) = 1 + z + z^2/2 + z^3/6 + z^4/24."""
    prob = _prob(n=2, N=4, p=3, flux="upwind")
    ops = dg2d.CartOps(prob)
    L = _dense_L(ops, prob)
    U, V = _rand_state(prob, 4)
    z = np.concatenate([U.ravel(), V.ravel()])
    dt = 0.1 * prob.hx
    A = dt * L
    expect = z + A @ z + A @ (A @ z) / 2 + A @ (A @ (A @ z)) / 6 + A @ (A @ (A @ (A @ z))) / 24
    U1, V1 = dg2d.rk4_step(U, V, dt, lambda a, b: dg2d.rhs(a, b, ops))
    np.testing.assert_allclose(np.concatenate([U1.ravel(), V1.ravel()]), expect, atol=1e-12)


@pytest.mark.parametrize("flux,N,p,cfl", [("central", 8, 3, 0.5), ("upwind", 8, 3, 0.2),
                                          ("upwind", 6, 5, 0.15)])
def test_spectrum_stable(flux, N, p, cfl):
    """Stability: Re(eig L) <= 0 (central: imaginary axis), |R4(dt lambda)| <= 1 at the CFL used."""
    prob = _prob(n=2, N=N, p=p, flux=flux)
    ops = dg2d.CartOps(prob)
    ev = np.linalg.eigvals(_dense_L(ops, prob))
    scale = np.abs(ev).max()
    assert ev.real.max() < 1e-6 * scale
    if flux == "central":
        assert np.abs(ev.real).max() < 1e-6 * scale
    z = cfl * prob.hx * (np.minimum(ev.real, 0) + 1j * ev.imag)
    assert np.abs(1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24).max() <= 1 + 1e-9


def test_standing_wave_config_small_and_fourth_order():
    """u = sin(2 pi x) sin(2 pi y) cos(2 sqrt(2) pi t) (4x4 elements, p = 3, central, CFL 0.5,
    t = 1): error ~1e-5 at N = 8 and observed order near p + 1 = 4 (paper, Sec. 6.2:
    2D rates 3.96-4.33 for p = 3)."""
    errs = []
    for N in (8, 16):
        prob = _prob(n=4, N=N, p=3, flux="central")
        ops = dg2d.CartOps(prob)
        X, Y = inputs.node_coords(4, 4, N)
        U, V = inputs.standing_wave(X, Y), np.zeros_like(X)
        dt = 0.5 * prob.hx
        U, V = dg2d.run(U, V, ops, dt, int(round(1.0 / dt)))
        ex = lambda x, y: np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.cos(2 * np.sqrt(2) * np.pi)
        errs.append(dg2d.l2_error(U, prob, ex))
    assert errs[0] < 5e-5
    rate = np.log2(errs[0] / errs[1])
    assert 3.5 < rate < 4.6, rate


def test_fourier_superposition_upwind_p5():
    """Exact solution of the periodic problem with v0 = 0:
    u = sum a_m cos(2 pi |k_m| t) cos(2 pi k_m.x + theta_m) (upwind, p = 5).  The bound is
    set by RK4's phase error, about (omega dt)^5 / 120 per step (omega dt ~ 0.08 here)."""
    n, N, p = 4, 12, 5
    prob = _prob(n=n, N=N, p=p, flux="upwind")
    ops = dg2d.CartOps(prob)
    modes = inputs.fourier_modes(7, n_modes=4, kmax=3)
    X, Y = inputs.node_coords(n, n, N)
    U, V = inputs.fourier_field(modes, X, Y), np.zeros_like(X)
    dt = 0.15 * prob.hx
    steps = 40
    U, V = dg2d.run(U, V, ops, dt, steps)
    T = dt * steps
    err = dg2d.l2_error(U, prob, lambda x, y: inputs.fourier_field(modes, x, y, t=T))
    ref = dg2d.l2_error(np.zeros_like(U), prob, lambda x, y: inputs.fourier_field(modes, x, y, t=T))
    assert err / ref < 1e-5, err / ref
