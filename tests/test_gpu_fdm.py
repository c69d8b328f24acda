"""GPU parity of the constant-coefficient path (simultaneous diagonalisation) against
the FP64 oracle, through the C ABI.

Bar: FP64 nodal state relative l2 <= 1e-12 against the oracle at t_final; FP32
storage mode <= 1e-6.  Sizes span several 4-element workgroup tiles with a ragged last
tile.
"""
import sys

import numpy as np
import pytest

from oracle import dg2d
from paper_2105_01722_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu(prob, U0, V0, dt, steps, precision="fp64"):
    from paper_2105_01722_amd import gdw
    s = gdw.Solver(prob.nx, prob.ny, prob.N, prob.p, c2=prob.c2, flux=prob.flux, xi=prob.xi,
                   precision=precision, Lx=prob.Lx, Ly=prob.Ly, x0=prob.x0, y0=prob.y0)
    s.set_state(U0, V0)
    s.run(dt, steps)
    U, V = s.get_state()
    E = s.energy()
    st = s.stats()
    s.close()
    return U.cpu().numpy(), V.cpu().numpy(), E, st


from _cmp import assert_close, rel as _rel, relmax as _relmax  # noqa: E402


def _lu_ops(prob):
    """Oracle operators with LU instead of Cholesky element solves: a second FP64 direct
    solver whose distance to the first measures the rounding floor of the problem."""
    import scipy.linalg as sla
    ops = dg2d.CartOps(prob)
    luS, luM = sla.lu_factor(ops.Shat), sla.lu_factor(ops.M2)

    def mk(lu):
        def solve(F):
            n = F.shape[0] * F.shape[1]
            return sla.lu_solve(lu, F.reshape(n, -1).T).T.reshape(F.shape)
        return solve
    ops.solve_Shat, ops.solve_M = mk(luS), mk(luM)
    return ops


def test_standing_wave_4x4_central_fp64():
    """4x4 elements, N = 8, p = 3, central, CFL 0.5, t = 1 (64 steps): oracle parity and
    the exact standing wave."""
    _say("case: standing wave 4x4 N8 p3 central fp64")
    prob = dg2d.CartProblem(nx=4, ny=4, N=8, p=3, flux="central")
    X, Y = inputs.node_coords(4, 4, 8)
    U0, V0 = inputs.standing_wave(X, Y), np.zeros_like(X)
    dt = 0.5 * prob.hx
    steps = int(round(1.0 / dt))
    Ug, Vg, Eg, st = _gpu(prob, U0, V0, dt, steps)
    ops = dg2d.CartOps(prob)
    Uo, Vo = dg2d.run(U0, V0, ops, dt, steps)
    assert_close(Ug, Uo, 1e-12)
    assert_close(Vg, Vo, 1e-12)
    Eo = dg2d.energy(Uo, Vo, ops)
    assert abs(Eg - Eo) <= 1e-13 * abs(Eo)
    E0 = dg2d.energy(U0, V0, ops)
    assert abs(Eg - E0) <= 1e-5 * E0        # RK4 drift only (central flux conserves)
    ex = lambda x, y: np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.cos(2 * np.sqrt(2) * np.pi)
    assert dg2d.l2_error(Ug, prob, ex) < 5e-5
    assert st["steps_taken"] == steps and st["dof_updates"] == steps * 16 * 81


@pytest.mark.parametrize("n,N,p,flux", [(3, 16, 5, "upwind"), (3, 12, 5, "upwind"),
                                        (5, 8, 3, "upwind"), (2, 16, 7, "upwind"),
                                        (3, 16, 5, "central")])
def test_fourier_modes_fp64(n, N, p, flux):
    """Seeded Fourier superposition, the specialised tile sizes N + 1 = 9, 13, 17."""
    _say("case: fourier", n, N, p, flux)
    prob = dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux=flux)
    X, Y = inputs.node_coords(n, n, N)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=4), X, Y)
    V0 = 0.3 * inputs.fourier_field(inputs.fourier_modes(3, kmax=4), X, Y)
    dt = 0.1 * prob.hx
    steps = 6
    Ug, Vg, _, _ = _gpu(prob, U0, V0, dt, steps)
    Uo, Vo = dg2d.run(U0, V0, dg2d.CartOps(prob), dt, steps)
    assert_close(Ug, Uo, 1e-12)
    assert_close(Vg, Vo, 1e-12)


@pytest.mark.parametrize("nx,ny,N,p,flux,c2", [(3, 2, 6, 3, "upwind", 2.0),
                                               (2, 3, 7, 5, "central", 0.6),
                                               (3, 3, 10, 7, "upwind", 1.3),
                                               (1, 1, 5, 5, "upwind", 1.0),
                                               (5, 3, 4, 1, "upwind", 1.0)])
def test_generic_sizes_rectangles_fp64(nx, ny, N, p, flux, c2):
    """Runtime-sized kernels, anisotropic elements (Lx/nx != Ly/ny), c^2 != 1, xi = c,
    a single element (self-neighbour through the periodic wrap) and p = 1.

    White-noise nodal data excites the top modes, where rounding is amplified by
    cond(S_hat) (1e6 at N = 10, p = 7).  The bar is therefore max(1e-12, 4 x the
    distance between two FP64 direct solvers of the oracle on the same input)."""
    _say("case: generic", nx, ny, N, p, flux, c2)
    prob = dg2d.CartProblem(nx=nx, ny=ny, N=N, p=p, flux=flux, c2=c2, Lx=1.3, Ly=0.7,
                            x0=-0.2, y0=0.1, xi=np.sqrt(c2))
    rng = np.random.default_rng(11)
    shp = (ny, nx, N + 1, N + 1)
    U0, V0 = rng.standard_normal(shp), rng.standard_normal(shp)
    dt = 0.05 * min(prob.hx, prob.hy)
    Ug, Vg, Eg, _ = _gpu(prob, U0, V0, dt, 5)
    ops = dg2d.CartOps(prob)
    Uo, Vo = dg2d.run(U0, V0, ops, dt, 5)
    U2, V2 = dg2d.run(U0, V0, _lu_ops(prob), dt, 5)
    tol_u = max(1e-12, 4 * _rel(U2, Uo))
    tol_v = max(1e-12, 4 * _rel(V2, Vo))
    assert_close(Ug, Uo, tol_u)
    assert_close(Vg, Vo, tol_v)
    Eo = dg2d.energy(Uo, Vo, ops)
    assert abs(Eg - Eo) <= 1e-12 * abs(Eo)


def test_zero_steps_roundtrip_and_constants():
    """set_state / get_state is the identity up to roundoff; constants stay constant."""
    _say("case: roundtrip")
    prob = dg2d.CartProblem(nx=3, ny=3, N=16, p=5, flux="upwind")
    rng = np.random.default_rng(5)
    U0 = rng.standard_normal((3, 3, 17, 17))
    Ug, Vg, _, _ = _gpu(prob, U0, -U0, 0.01, 0)
    assert _rel(Ug, U0) < 1e-13 and _rel(Vg, -U0) < 1e-13
    C = np.full((3, 3, 17, 17), 2.5)
    Ug, Vg, _, _ = _gpu(prob, C, np.zeros_like(C), 0.1 * prob.hx, 10)
    assert np.abs(Ug - 2.5).max() < 1e-11 and np.abs(Vg).max() < 1e-9


@pytest.mark.parametrize("flux", ["upwind", "central"])
def test_fp32_mode_within_1e6(flux):
    """FP32 storage of the stage increments around the FP64 register y: U and V within
    1e-6 of the FP64 oracle, in relative l2 and in relative element-wise max (the same
    bar for both; measured about 1e-9 here)."""
    _say("case: fp32", flux)
    n, N, p = 6, 16, 5
    prob = dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux=flux)
    X, Y = inputs.node_coords(n, n, N)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=6), X, Y)
    V0 = 3.0 * inputs.fourier_field(inputs.fourier_modes(3, kmax=6), X, Y)
    dt = 0.15 * prob.hx
    steps = 20
    Ug, Vg, Eg, _ = _gpu(prob, U0, V0, dt, steps, precision="fp32")
    ops = dg2d.CartOps(prob)
    Uo, Vo = dg2d.run(U0, V0, ops, dt, steps)
    _say("  rel l2 U %.2e V %.2e, max U %.2e V %.2e" % (
        _rel(Ug, Uo), _rel(Vg, Vo), _relmax(Ug, Uo), _relmax(Vg, Vo)))
    assert_close(Ug, Uo, 1e-6, max_bar=1e-6)
    assert_close(Vg, Vo, 1e-6, max_bar=1e-6)
    Eo = dg2d.energy(Uo, Vo, ops)
    assert abs(Eg - Eo) <= 1e-6 * abs(Eo)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nonfinite_state_reported(precision):
    """A NaN in the initial data propagates through the arithmetic (every kernel still runs
    to completion) and the end-of-run check reports it: gdw_get_stats and gdw_energy return
    ENONFINITE, and the context stays usable (a finite state set afterwards runs clean)."""
    _say("case: nonfinite state", precision)
    from paper_2105_01722_amd import gdw
    prob = dg2d.CartProblem(nx=3, ny=2, N=8, p=3, flux="upwind")
    rng = np.random.default_rng(5)
    U0 = rng.standard_normal((2, 3, 9, 9))
    V0 = rng.standard_normal((2, 3, 9, 9))
    bad = U0.copy()
    bad[1, 2, 4, 4] = np.nan
    s = gdw.Solver(prob.nx, prob.ny, prob.N, prob.p, c2=prob.c2, flux=prob.flux, xi=prob.xi,
                   precision=precision, Lx=prob.Lx, Ly=prob.Ly, x0=prob.x0, y0=prob.y0)
    try:
        s.set_state(bad, V0)
        s.run(0.1 * prob.hx, 2)
        st = s.stats(check=False)
        assert st["status"] == gdw.GDW_ENONFINITE
        with pytest.raises(gdw.GdwError) as ei:
            s.energy()
        assert ei.value.status == gdw.GDW_ENONFINITE
        s.set_state(U0, V0)
        s.run(0.1 * prob.hx, 2)
        assert s.stats(check=False)["status"] == gdw.GDW_OK
        assert np.isfinite(s.energy())
    finally:
        s.close()


@pytest.mark.parametrize("nx,ny,N,p,precision,bc", [
    (2, 3, 31, 7, "fp64", ("periodic",) * 4),      # N + 1 = 32: 1024 threads, 2 elements per tile
    (3, 2, 31, 5, "fp32", ("periodic",) * 4),
    (3, 2, 5, 5, "fp64", ("periodic",) * 4),       # N = p
    (2, 2, 7, 7, "fp64", ("dirichlet",) * 4),
    (1, 1, 9, 3, "fp64", ("dirichlet", "dirichlet", "neumann", "neumann")),  # one element, walls
])
def test_largest_and_degenerate_sizes(nx, ny, N, p, precision, bc):
    """The largest element the library accepts (N + 1 = 32, one thread per modal index:
    1024 threads, the workgroup limit), the smallest N for a degree (N = p), and a single
    element whose four faces are all walls.  Smooth data.  FP64 bar: max(1e-12, 4 x the
    oracle's Cholesky-vs-LU spread, 4 x the distance between the oracle with S and with
    S~ = M Psi Lambda Psi^T M from an FP64 eigenbasis) -- the rounding floor of a
    simultaneous-diagonalisation solve, which grows with cond(S_hat) and is largest at
    N + 1 = 32, p = 7."""
    _say("case: extreme sizes", nx, ny, N, p, precision, bc)
    from paper_2105_01722_amd import gdw
    prob = dg2d.CartProblem(nx=nx, ny=ny, N=N, p=p, flux="upwind", bc=bc)
    X, Y = dg2d.node_coords(prob)
    U0 = inputs.fourier_field(inputs.fourier_modes(6, kmax=3), X, Y)
    V0 = 0.2 * inputs.fourier_field(inputs.fourier_modes(7, kmax=3), X, Y)
    dt = 0.05 * prob.hx
    s = gdw.Solver(nx, ny, N, p, flux="upwind", xi=1.0, precision=precision, bc=bc)
    try:
        s.set_state(U0, V0)
        s.run(dt, 4)
        Ug, Vg = (x.cpu().numpy() for x in s.get_state())
        assert s.stats()["status"] == 0
    finally:
        s.close()
    Uo, Vo = dg2d.run(U0, V0, dg2d.CartOps(prob), dt, 4)
    if precision == "fp32":
        assert_close(Ug, Uo, 1e-6)
        return
    from test_gpu_fullsize import _eigen_ops
    U2, V2 = dg2d.run(U0, V0, _lu_ops(prob), dt, 4)
    U3, V3 = dg2d.run(U0, V0, _eigen_ops(dg2d.CartOps(prob)), dt, 4)
    _say("  rel U %.1e (lu %.1e, S~ %.1e)" % (_rel(Ug, Uo), _rel(U2, Uo), _rel(U3, Uo)))
    assert_close(Ug, Uo, max(1e-12, 4 * _rel(U2, Uo), 4 * _rel(U3, Uo)))
    assert_close(Vg, Vo, max(1e-12, 4 * _rel(V2, Vo), 4 * _rel(V3, Vo)))