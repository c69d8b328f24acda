"""Pins of the wall boundaries of the oracle (constant-coefficient and mapped paths).

The paper gives no boundary flux; its 2D Dirichlet experiment (Sec. 6, "Dirichlet
Boundary Conditions in Two Dimensions") has homogeneous Dirichlet data on the unit
square.  The oracle's reading: a wall face uses the interior flux of Sec. 2.2.1 with a
mirror exterior state (Dirichlet: the odd mirror, Neumann: the even mirror).

What fixes it independently of its own code:
  * reflection: on a GD grid the basis of an element maps to itself under x -> -x, so
    the scheme on [0, L] with a Dirichlet (Neumann) wall is the periodic scheme on
    [-L, L] with odd (even) data -- the periodic scheme being pinned by the printed 1D
    rate tables (test_oracle_convergence.py).  A wrong sign of either mirrored trace,
    or a mirror taken from the wrong face, breaks the identity;
  * energy: with the central flux the discrete energy of Sec. 2.2 is conserved with
    walls too (dE/dt = 0), with the upwind flux it does not grow;
  * a Dirichlet standing wave sin(k pi x) sin(l pi y) cos(omega t) keeps zero boundary
    values and converges to the exact solution;
  * mapped path: on an affine mesh it is the Cartesian wall scheme; on a curved mesh with
    variable c^2 the energy identity holds with walls (wall faces dissipate against the
    mirror state with half weight).
"""
import numpy as np
import pytest

from oracle import dg2d, general
from paper_2105_01722_amd import inputs


def _odd_even_extend(W, axis_x, axis_y):
    """Extend a field [ny, nx, n1, n1] across the W side (x) and the S side (y).

    axis_x / axis_y: None (no extension), +1 (even mirror) or -1 (odd mirror).  The mirror
    of element ex is element nx - 1 - ex of the new left half, its node ix is N - ix."""
    if axis_x is not None:
        W = np.concatenate([axis_x * W[:, ::-1, :, ::-1], W], axis=1)
    if axis_y is not None:
        W = np.concatenate([axis_y * W[::-1, :, ::-1, :], W], axis=0)
    return W


def _pair(bc, n=(3, 2), N=6, p=3, flux="upwind", c2=1.3, L=(1.0, 0.7)):
    """Wall problem on [0, Lx] x [0, Ly] and the periodic problem on the doubled domain."""
    nx, ny = n
    kind = {"dirichlet": -1.0, "neumann": 1.0, "periodic": None}
    sx, sy = kind[bc[1]], kind[bc[3]]       # W and S sides carry the mirror
    wall = dg2d.CartProblem(nx=nx, ny=ny, N=N, p=p, flux=flux, c2=c2, xi=np.sqrt(c2),
                            Lx=L[0], Ly=L[1], bc=bc)
    per = dg2d.CartProblem(nx=nx * (2 if sx else 1), ny=ny * (2 if sy else 1), N=N, p=p,
                           flux=flux, c2=c2, xi=np.sqrt(c2),
                           Lx=L[0] * (2 if sx else 1), Ly=L[1] * (2 if sy else 1),
                           x0=-L[0] if sx else 0.0, y0=-L[1] if sy else 0.0)
    return wall, per, sx, sy


def _restrict(W, nx, ny):
    return W[-ny:, -nx:]


@pytest.mark.parametrize("bc", [
    ("dirichlet",) * 4,
    ("neumann",) * 4,
    ("dirichlet", "dirichlet", "neumann", "neumann"),
    ("periodic", "periodic", "dirichlet", "dirichlet"),
    ("neumann", "neumann", "periodic", "periodic"),
])
@pytest.mark.parametrize("flux", ["central", "upwind"])
def test_wall_is_the_mirrored_periodic_scheme(bc, flux):
    wall, per, sx, sy = _pair(bc, flux=flux)
    ow, op = dg2d.CartOps(wall), dg2d.CartOps(per)
    rng = np.random.default_rng(7)
    shp = (wall.ny, wall.nx, wall.N + 1, wall.N + 1)
    U, V = rng.standard_normal(shp), rng.standard_normal(shp)
    du, dv = dg2d.rhs(U, V, ow)
    Ue, Ve = _odd_even_extend(U, sx, sy), _odd_even_extend(V, sx, sy)
    due, dve = dg2d.rhs(Ue, Ve, op)
    scale = max(np.abs(due).max(), np.abs(dve).max())
    assert np.abs(_restrict(due, wall.nx, wall.ny) - du).max() <= 1e-12 * scale
    assert np.abs(_restrict(dve, wall.nx, wall.ny) - dv).max() <= 1e-12 * scale
    # the periodic evolution keeps the mirror symmetry
    assert np.abs(_odd_even_extend(du, sx, sy) - due).max() <= 1e-12 * scale
    # and a few RK4 steps agree as well
    dt = 0.1 * wall.hx
    Uw, Vw = dg2d.run(U, V, ow, dt, 3)
    Up, Vp = dg2d.run(Ue, Ve, op, dt, 3)
    assert np.abs(_restrict(Up, wall.nx, wall.ny) - Uw).max() <= 1e-12 * np.abs(Up).max()


def test_wrong_mirror_sign_breaks_the_identity():
    """The identity above is sharp: flipping the sign of the mirrored derivative (the
    Neumann state on a Dirichlet wall) changes the right-hand side at order one."""
    bc = ("dirichlet",) * 4
    wall, per, sx, sy = _pair(bc)
    rng = np.random.default_rng(8)
    shp = (wall.ny, wall.nx, wall.N + 1, wall.N + 1)
    U, V = rng.standard_normal(shp), rng.standard_normal(shp)
    wrong = dg2d.CartProblem(**{**wall.__dict__, "bc": ("neumann",) * 4})
    du, _ = dg2d.rhs(U, V, dg2d.CartOps(wrong))
    due, _ = dg2d.rhs(_odd_even_extend(U, sx, sy), _odd_even_extend(V, sx, sy),
                      dg2d.CartOps(per))
    assert np.abs(_restrict(due, wall.nx, wall.ny) - du).max() > 1e-3 * np.abs(due).max()


@pytest.mark.parametrize("bc", [("dirichlet",) * 4, ("neumann",) * 4,
                                ("neumann", "neumann", "dirichlet", "dirichlet")])
def test_energy_with_walls(bc):
    """Central flux: dE/dt = 0 with walls; upwind: dE/dt < 0 for generic data."""
    rng = np.random.default_rng(9)
    for flux in ("central", "upwind"):
        prob = dg2d.CartProblem(nx=3, ny=3, N=7, p=5, flux=flux, c2=0.8, xi=np.sqrt(0.8),
                                bc=bc)
        ops = dg2d.CartOps(prob)
        U = rng.standard_normal((3, 3, 8, 8))
        V = rng.standard_normal((3, 3, 8, 8))
        rate = dg2d.energy_rate(U, V, ops)
        E = dg2d.energy(U, V, ops)
        if flux == "central":
            assert abs(rate) <= 1e-12 * E
        else:
            assert rate < -1e-6 * E


def test_dirichlet_standing_wave_converges():
    """u = cos(sqrt(2) pi t) sin(pi x) sin(pi y) on the unit square with Dirichlet walls:
    the nodal error at t = 0.25 falls by about 2^(p+1) when h halves (p = 3)."""
    errs = []
    for n in (2, 4):
        prob = dg2d.CartProblem(nx=n, ny=n, N=6, p=3, flux="upwind", bc=("dirichlet",) * 4)
        ops = dg2d.CartOps(prob)
        X, Y = dg2d.node_coords(prob)
        U0 = np.sin(np.pi * X) * np.sin(np.pi * Y)
        V0 = np.zeros_like(U0)
        steps = 8 * n
        T = 0.25
        U, V = dg2d.run(U0, V0, ops, T / steps, steps)
        exact = np.cos(np.sqrt(2.0) * np.pi * T) * U0
        errs.append(dg2d.l2_error(U, prob, lambda x, y: np.cos(np.sqrt(2.0) * np.pi * T)
                                  * np.sin(np.pi * x) * np.sin(np.pi * y)))
        assert np.abs(U - exact).max() < 1e-3
    rate = np.log2(errs[0] / errs[1])
    assert rate > 3.3, (errs, rate)


# ---- walls on the mapped / variable-coefficient oracle -------------------------------


@pytest.mark.parametrize("bc", [("dirichlet",) * 4, ("neumann", "neumann", "dirichlet", "dirichlet"),
                                ("periodic", "periodic", "neumann", "neumann")])
@pytest.mark.parametrize("flux", ["central", "upwind"])
def test_general_walls_on_affine_mesh_equal_cartesian_walls(bc, flux):
    """The quadrature-based general oracle on a rectangle grid with constant c^2 and walls
    is the Cartesian wall scheme (the mirror is taken at the face points there)."""
    n, N, p, c2 = 3, 6, 3, 1.7
    X, Y = inputs.node_coords(n, n, N, Lx=1.3, Ly=0.7, x0=-0.2, y0=0.1)
    g = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux=flux, xi=np.sqrt(c2),
                                          bc=bc), X, Y, np.full_like(X, c2))
    c = dg2d.CartOps(dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux=flux, c2=c2, xi=np.sqrt(c2),
                                      Lx=1.3, Ly=0.7, x0=-0.2, y0=0.1, bc=bc))
    rng = np.random.default_rng(2)
    U, V = rng.standard_normal(X.shape), rng.standard_normal(X.shape)
    for x, y in zip(general.rhs(U, V, g), dg2d.rhs(U, V, c)):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(y).max()


@pytest.mark.parametrize("bc", [("dirichlet",) * 4, ("neumann",) * 4,
                                ("dirichlet", "dirichlet", "neumann", "neumann")])
def test_general_walls_energy_identity_curved_variable(bc):
    """Curved mesh (the walls stay straight: the mapping's displacement vanishes on the
    sides of the unit square) and variable c^2: central conserves the energy exactly;
    upwind dissipates exactly the face integral, every face of every element taken with
    weight 1/2 (interior faces once, wall faces half, against the mirror state)."""
    n, N, p = 3, 6, 3
    X, Y = inputs.node_coords(n, n, N)
    Xm, Ym = inputs.mapped_coords(X, Y)
    c2 = inputs.c2_field(3, X, Y)
    rng = np.random.default_rng(3)
    U, V = rng.standard_normal(X.shape), rng.standard_normal(X.shape)
    ne = n * n
    for flux in ("central", "upwind"):
        g = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux=flux, bc=bc), Xm, Ym, c2)
        dU, dV = general.rhs(U, V, g)
        rate = (np.einsum("ei,eij,ej->", V.reshape(ne, -1), g.M, dV.reshape(ne, -1))
                + np.einsum("ei,eij,ej->", U.reshape(ne, -1), g.S, dU.reshape(ne, -1)))
        scale = np.abs(np.einsum("ei,eij,ej->e", V.reshape(ne, -1), g.M, dV.reshape(ne, -1))).sum()
        if flux == "central":
            assert abs(rate) < 1e-11 * scale
        else:
            d = general.face_dissipation(U, V, g)
            assert d < 0 and abs(rate - d) < 1e-11 * abs(d)
