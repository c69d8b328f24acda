"""Pins of the source term f of the constant-coefficient oracle (Sec. 2: u_tt =
div(c^2 grad u) + f), with f = sum_k sin(omega_k t + phase_k) g_k(x, y) represented by
the GD interpolant of each g_k.

What fixes it: a manufactured solution (the exact solution of the forced PDE) converges
at the design order, which a wrong sign, scale or stage time of the term would destroy;
and the discrete energy balance with the central flux is exactly the work of the source,
dE/dt = sum_k s_k(t) V^T M g_k.
"""
import numpy as np
import pytest

from oracle import dg2d

OMEGA = 5.0


def _manufactured(n, N, p, c2, bc=("periodic",) * 4, k=2.0):
    """u = sin(omega t) sin(k pi x) sin(k pi y): f = (2 (k pi)^2 c^2 - omega^2) sin(omega t) g
    with g = sin(k pi x) sin(k pi y); u(0) = 0, v(0) = omega g."""
    base = dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux="upwind", c2=c2, xi=np.sqrt(c2), bc=bc)
    X, Y = dg2d.node_coords(base)
    g = np.sin(k * np.pi * X) * np.sin(k * np.pi * Y)
    amp = 2.0 * (k * np.pi) ** 2 * c2 - OMEGA ** 2
    prob = dg2d.CartProblem(**{**base.__dict__, "forcing": ((amp * g, OMEGA, 0.0),)})
    return prob, g


@pytest.mark.parametrize("bc,k", [(("periodic",) * 4, 2.0), (("dirichlet",) * 4, 1.0)])
def test_manufactured_solution_converges(bc, k):
    T = 0.3
    errs = []
    for n in (2, 4):
        prob, g = _manufactured(n, 6, 3, 1.3, bc, k)
        ops = dg2d.CartOps(prob)
        steps = 12 * n
        U, V = dg2d.run(np.zeros_like(g), OMEGA * g, ops, T / steps, steps)
        exact = np.sin(OMEGA * T) * g
        errs.append(dg2d.l2_error(U, prob, lambda x, y: np.sin(OMEGA * T)
                                  * np.sin(k * np.pi * x) * np.sin(k * np.pi * y)))
        assert np.abs(U - exact).max() < 2e-2 * np.abs(exact).max()
    rate = np.log2(errs[0] / errs[1])
    assert rate > 3.3, (errs, rate)


def test_run_split_in_two_calls_keeps_the_clock():
    """run(..., t0) continues the source's clock: 6 steps = 4 steps + 2 steps from t0."""
    prob, g = _manufactured(2, 6, 3, 1.3)
    ops = dg2d.CartOps(prob)
    dt = 0.01
    U1, V1 = dg2d.run(np.zeros_like(g), OMEGA * g, ops, dt, 6)
    Ua, Va = dg2d.run(np.zeros_like(g), OMEGA * g, ops, dt, 4)
    U2, V2 = dg2d.run(Ua, Va, ops, dt, 2, t0=4 * dt)
    assert np.abs(U1 - U2).max() <= 1e-14 * np.abs(U1).max()


def test_energy_balance_is_the_work_of_the_source():
    """Central flux: dE/dt = sum_k s_k(t) V^T M g_k for any state and time."""
    rng = np.random.default_rng(4)
    n, N, p = 3, 7, 5
    base = dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux="central", c2=0.9)
    shp = (n, n, N + 1, N + 1)
    g1, g2 = rng.standard_normal(shp), rng.standard_normal(shp)
    prob = dg2d.CartProblem(**{**base.__dict__, "forcing": ((g1, 3.0, 0.2), (g2, 7.0, -1.0))})
    ops = dg2d.CartOps(prob)
    U, V = rng.standard_normal(shp), rng.standard_normal(shp)
    t = 0.37
    dU, dV = dg2d.rhs(U, V, ops, t)
    ne = n * n
    u, v = U.reshape(ne, -1), V.reshape(ne, -1)
    du, dv = dU.reshape(ne, -1), dV.reshape(ne, -1)
    dE = (np.einsum("ei,ij,ej->", v, ops.M2, dv)
          + prob.c2 * np.einsum("ei,ij,ej->", u, ops.S2, du))
    work = sum(np.sin(w * t + ph) * np.einsum("ei,ij,ej->", v, ops.M2, gk.reshape(ne, -1))
               for gk, w, ph in prob.forcing)
    assert abs(dE - work) <= 1e-11 * abs(work)


# ---- the mapped / variable-coefficient oracle ----------------------------------------
def _curved_manufactured(n, N, p):
    """u = sin(omega t) phi, phi = sin(2 pi x) sin(2 pi y) on the curved mesh, with
    c^2 = 1 + 0.25 sin(2 pi x) cos(2 pi y):  f = sin(omega t) (-omega^2 phi
    - c^2 lap(phi) - grad(c^2) . grad(phi)), everything at the physical nodes."""
    from oracle import general
    from paper_2105_01722_amd import inputs
    X, Y = inputs.node_coords(n, n, N)
    Xm, Ym = inputs.mapped_coords(X, Y)
    tp = 2 * np.pi
    phi = np.sin(tp * Xm) * np.sin(tp * Ym)
    c2 = 1.0 + 0.25 * np.sin(tp * Xm) * np.cos(tp * Ym)
    c2x = 0.25 * tp * np.cos(tp * Xm) * np.cos(tp * Ym)
    c2y = -0.25 * tp * np.sin(tp * Xm) * np.sin(tp * Ym)
    phx = tp * np.cos(tp * Xm) * np.sin(tp * Ym)
    phy = tp * np.sin(tp * Xm) * np.cos(tp * Ym)
    g = -OMEGA ** 2 * phi + 2 * tp ** 2 * c2 * phi - (c2x * phx + c2y * phy)
    prob = general.GenProblem(nx=n, ny=n, N=N, p=p, flux="upwind", forcing=((g, OMEGA, 0.0),))
    return general.GenOps(prob, Xm, Ym, c2), phi


def test_curved_variable_manufactured_solution_converges():
    """The exact solution of the forced variable-coefficient PDE on a curved mesh: the
    nodal error at t = 0.2 falls at about the design order (> 3.3 for p = 3) when h halves;
    a wrong metric term or coefficient gradient in the operator would stop it at O(1)."""
    from oracle import general
    T = 0.2
    errs = []
    for n in (2, 4):
        ops, phi = _curved_manufactured(n, 6, 3)
        steps = 10 * n
        U, V = general.run(np.zeros_like(phi), OMEGA * phi, ops, T / steps, steps)
        errs.append(np.abs(U - np.sin(OMEGA * T) * phi).max())
    rate = np.log2(errs[0] / errs[1])
    assert errs[1] < 2e-3 and rate > 3.3, (errs, rate)
