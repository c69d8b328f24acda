"""Pins of the mapped / variable-coefficient oracle (Sec. 2.2 weak form, Sec. 7).

What fixes the answer: the Cartesian constant-coefficient case of Sec. 3 (the
quadrature assembly must reproduce the Kronecker operators), the energy identity
of DG1 / DG2 (central: conserved; upwind: the face dissipation integral), exact
preservation of constants on curved meshes, and exact travelling-wave solutions on
a curved mesh (c = 1: the mesh changes, the PDE does not) with the design order.
"""
import numpy as np
import pytest

from oracle import dg2d, general
from paper_2105_01722_amd import inputs


def _mapped(n, N, seed=3):
    X, Y = inputs.node_coords(n, n, N)
    Xm, Ym = inputs.mapped_coords(X, Y)
    return X, Y, Xm, Ym, inputs.c2_field(seed, X, Y)


@pytest.mark.parametrize("flux", ["central", "upwind"])
def test_affine_map_reproduces_cartesian(flux):
    """A rectangle grid (Hx != Hy) with constant c^2 is the Cartesian case of Sec. 3."""
    n, N, p, c2 = 3, 6, 3, 1.7
    X, Y = inputs.node_coords(n, n, N, Lx=1.3, Ly=0.7, x0=-0.2, y0=0.1)
    gp = general.GenProblem(nx=n, ny=n, N=N, p=p, flux=flux, xi=np.sqrt(c2))
    g = general.GenOps(gp, X, Y, np.full_like(X, c2))
    cp = dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux=flux, c2=c2, xi=np.sqrt(c2),
                          Lx=1.3, Ly=0.7, x0=-0.2, y0=0.1)
    c = dg2d.CartOps(cp)
    np.testing.assert_allclose(g.M[4], c.M2, atol=1e-16)
    np.testing.assert_allclose(g.S[4], c2 * c.S2, atol=1e-12)
    rng = np.random.default_rng(0)
    U, V = rng.standard_normal(X.shape), rng.standard_normal(X.shape)
    a, b = general.rhs(U, V, g), dg2d.rhs(U, V, c)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(y).max()


@pytest.mark.parametrize("p,N", [(3, 6), (5, 7)])
def test_energy_identity_mapped_variable(p, N):
    """DG1 / DG2 with test functions U, V: central conserves energy exactly, upwind
    dissipates exactly the face integral of c^2 (beta (a + a_nb)^2 + tau (v_nb - v)^2)."""
    n = 3
    X, Y, Xm, Ym, c2 = _mapped(n, N)
    rng = np.random.default_rng(1)
    U, V = rng.standard_normal(X.shape), rng.standard_normal(X.shape)
    for flux in ("central", "upwind"):
        g = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux=flux), Xm, Ym, c2)
        dU, dV = general.rhs(U, V, g)
        ne = n * n
        rate = (np.einsum("ei,eij,ej->", V.reshape(ne, -1), g.M, dV.reshape(ne, -1))
                + np.einsum("ei,eij,ej->", U.reshape(ne, -1), g.S, dU.reshape(ne, -1)))
        scale = np.abs(np.einsum("ei,eij,ej->e", V.reshape(ne, -1), g.M, dV.reshape(ne, -1))).sum()
        if flux == "central":
            assert abs(rate) < 1e-11 * scale
        else:
            d = general.face_dissipation(U, V, g)
            assert d < 0 and abs(rate - d) < 1e-11 * abs(d)


def test_constants_preserved_on_curved_mesh():
    """Free-stream preservation: constant u with v = 0 is steady; constant v translates u."""
    n, N, p = 3, 7, 5
    X, Y, Xm, Ym, c2 = _mapped(n, N)
    g = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="upwind"), Xm, Ym, c2)
    C = np.full(X.shape, 2.0)
    dU, dV = general.rhs(C, 0 * C, g)
    # rounding bound for dV = M^{-1}(-S 1 * 2): ~ n eps ||S|| |u| / lambda_min(M)
    lmin = min(np.linalg.eigvalsh(m).min() for m in g.M)
    bound = 1e3 * np.finfo(float).eps * np.abs(g.S).max() * 2.0 / lmin
    assert np.abs(dU).max() < 1e-12 and np.abs(dV).max() < bound
    dU, dV = general.rhs(0 * C, C, g)
    assert np.abs(dU - 2.0).max() < 1e-11 and np.abs(dV).max() < 1e-11


def test_element_matrices_structure():
    """M_J SPD; S_K symmetric positive semi-definite with the constants as null space;
    S_hat SPD; w sums to the element area int J."""
    n, N, p = 2, 6, 3
    X, Y, Xm, Ym, c2 = _mapped(n, N)
    g = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p), Xm, Ym, c2)
    for e in range(n * n):
        np.testing.assert_allclose(g.M[e], g.M[e].T, atol=1e-16)
        np.testing.assert_allclose(g.S[e], g.S[e].T, atol=1e-11)
        assert np.linalg.eigvalsh(g.M[e]).min() > 0
        ev = np.linalg.eigvalsh(g.S[e])
        assert ev[0] > -1e-10 and ev[1] > 1e-6
        assert np.abs(g.S[e] @ np.ones(g.n1 ** 2)).max() < 1e-10
        assert np.linalg.eigvalsh(g.Shat[e]).min() > 0
    np.testing.assert_allclose(g.area.sum(), 1.0, atol=1e-12)   # the map is onto the unit square


def test_travelling_wave_on_curved_mesh_converges():
    """c = 1 on the mapped mesh: u = cos(2 pi (x + y) - 2 sqrt(2) pi t) solves the problem;
    the error at the nodes (physical coordinates) falls at about the design order p+1."""
    p, n, T = 3, 4, 0.05
    errs = []
    for N in (6, 12):
        X, Y = inputs.node_coords(n, n, N)
        Xm, Ym = inputs.mapped_coords(X, Y)
        g = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="upwind"),
                           Xm, Ym, np.ones_like(X))
        k = 2 * np.pi
        w = k * np.sqrt(2.0)
        U = np.cos(k * (Xm + Ym))
        V = w * np.sin(k * (Xm + Ym))
        h = 1.0 / (n * N)
        steps = int(np.ceil(T / (0.1 * h)))
        dt = T / steps
        U1, _ = general.run(U, V, g, dt, steps)
        ex = np.cos(k * (Xm + Ym) - w * T)
        errs.append(np.abs(U1 - ex).max())
    rate = np.log2(errs[0] / errs[1])
    assert errs[1] < 2e-4 and rate > 3.7, (errs, rate)
