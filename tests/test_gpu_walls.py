"""GPU parity of wall boundaries (Dirichlet / Neumann mirror states) on the
constant-coefficient path and on the PCG path (mapped elements, variable c^2), through
the C ABI, and the paper's 2D Dirichlet experiment.

Parity bar: FP64 nodal state relative l2 <= 1e-12 against the FP64 oracle (the same bar
as the periodic tests), FP32 storage <= 1e-6.  Grids span several 4-element workgroup
tiles with a ragged last tile, and put wall faces on both ends of tiles and inside them.

The second part runs the experiment of Sec. 6 "Dirichlet Boundary Conditions in Two
Dimensions" on the GPU path and compares the regression rates with the printed ones
(tests/golden/rates_2d_dirichlet.txt), with the bars of the 1D periodic pin
(test_oracle_convergence.py): energy-norm rates within 0.25, L2 rates within 0.6 for
p = 3 and 5.  Not compared, as there: p = 1 (order reduction, erratic in the range), and
the L2 rate at p = 7, which depends most on the range of h used for the regression (the
paper gives its grids only in a figure); on these grids it comes within 0.65 of the
printed values.
"""
import os
import sys

import numpy as np
import pytest

from oracle import dg2d, gd1d, general
from paper_2105_01722_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rates_2d_dirichlet.txt")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


from _cmp import assert_close, rel as _rel, relmax as _relmax  # noqa: E402


def _gpu(prob, U0, V0, dt, steps, precision="fp64"):
    from paper_2105_01722_amd import gdw
    s = gdw.Solver(prob.nx, prob.ny, prob.N, prob.p, c2=prob.c2, flux=prob.flux, xi=prob.xi,
                   precision=precision, Lx=prob.Lx, Ly=prob.Ly, x0=prob.x0, y0=prob.y0,
                   bc=prob.bc)
    try:
        s.set_state(U0, V0)
        s.run(dt, steps)
        U, V = s.get_state()
        E = s.energy()
        st = s.stats()
    finally:
        s.close()
    return U.cpu().numpy(), V.cpu().numpy(), E, st


BCS = {
    "dirichlet": ("dirichlet",) * 4,
    "neumann": ("neumann",) * 4,
    "mixed": ("dirichlet", "dirichlet", "neumann", "neumann"),
    "x_periodic": ("periodic", "periodic", "dirichlet", "dirichlet"),
    "y_periodic": ("neumann", "neumann", "periodic", "periodic"),
}


@pytest.mark.parametrize("bcname", list(BCS))
@pytest.mark.parametrize("nx,ny,N,p,flux", [(5, 3, 8, 3, "upwind"), (7, 2, 12, 5, "central"),
                                            (3, 3, 16, 5, "upwind"), (2, 5, 10, 7, "upwind")])
def test_walls_match_oracle_fp64(bcname, nx, ny, N, p, flux):
    _say("case: walls fp64", bcname, nx, ny, N, p, flux)
    prob = dg2d.CartProblem(nx=nx, ny=ny, N=N, p=p, flux=flux, c2=1.3, xi=np.sqrt(1.3),
                            Lx=1.2, Ly=0.8, x0=-0.1, y0=0.2, bc=BCS[bcname])
    X, Y = dg2d.node_coords(prob)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=4), X, Y)
    V0 = 0.3 * inputs.fourier_field(inputs.fourier_modes(3, kmax=4), X, Y)
    dt = 0.1 * min(prob.hx, prob.hy)
    steps = 6
    Ug, Vg, Eg, st = _gpu(prob, U0, V0, dt, steps)
    ops = dg2d.CartOps(prob)
    Uo, Vo = dg2d.run(U0, V0, ops, dt, steps)
    assert_close(Ug, Uo, 1e-12)
    assert_close(Vg, Vo, 1e-12)
    Eo = dg2d.energy(Uo, Vo, ops)
    assert abs(Eg - Eo) <= 1e-12 * abs(Eo)
    assert st["status"] == 0


@pytest.mark.parametrize("bcname", ["dirichlet", "mixed"])
def test_walls_fp32_within_1e6(bcname):
    _say("case: walls fp32", bcname)
    prob = dg2d.CartProblem(nx=9, ny=3, N=12, p=5, flux="upwind", bc=BCS[bcname])
    X, Y = dg2d.node_coords(prob)
    U0 = inputs.fourier_field(inputs.fourier_modes(4, kmax=4), X, Y)
    V0 = np.zeros_like(U0)
    dt = 0.1 * prob.hx
    Ug, Vg, _, _ = _gpu(prob, U0, V0, dt, 8, precision="fp32")
    Uo, Vo = dg2d.run(U0, V0, dg2d.CartOps(prob), dt, 8)
    assert_close(Ug, Uo, 1e-6)


def test_dirichlet_keeps_odd_symmetry_of_the_doubled_periodic_run():
    """The GPU wall run equals the GPU periodic run on the doubled domain with odd data
    (the reflection identity pinned for the oracle), here without the oracle."""
    _say("case: walls vs doubled periodic")
    n, N, p = 3, 8, 3
    wall = dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux="upwind", bc=BCS["dirichlet"])
    per = dg2d.CartProblem(nx=2 * n, ny=2 * n, N=N, p=p, flux="upwind", Lx=2.0, Ly=2.0,
                           x0=-1.0, y0=-1.0)
    rng = np.random.default_rng(12)
    U0 = rng.standard_normal((n, n, N + 1, N + 1))
    V0 = rng.standard_normal((n, n, N + 1, N + 1))

    def odd(W):
        W = np.concatenate([-W[:, ::-1, :, ::-1], W], axis=1)
        return np.concatenate([-W[::-1, :, ::-1, :], W], axis=0)

    dt = 0.1 * wall.hx
    Uw, _, _, _ = _gpu(wall, U0, V0, dt, 4)
    Up, _, _, _ = _gpu(per, odd(U0), odd(V0), dt, 4)
    assert np.abs(Up[-n:, -n:] - Uw).max() <= 1e-11 * np.abs(Up).max()


# ---- the paper's 2D Dirichlet experiment ----------------------------------------------
K = 15.0 * np.pi
OMEGA = np.sqrt(2.0) * K
T_FINAL = 0.2
CFL = 0.075 / (2.0 * np.pi)
GRIDS = {
    "Nfixed": [(n, 10) for n in (8, 10, 12, 16, 20, 24, 32)],
    "nfixed": [(10, N) for N in (10, 12, 14, 16, 20, 24)],
}


def _golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            table, flux, p, r_l2, r_en = line.split()
            out[(table, flux, int(p))] = (float(r_l2), float(r_en))
    return out


def _errors(U, V, prob, t):
    """L2 error of u and energy-norm error at time t, (p+3)-point Gauss quadrature per
    cell of the GD interpolants (the error measures of Sec. 6)."""
    N, p = prob.N, prob.p
    xg, wg = gd1d.gauss_legendre(p + 3)
    tq = (np.arange(N)[:, None] + xg[None, :]).ravel()
    wq = np.tile(wg, N)
    B, dB = gd1d.basis_eval(N, p, tq)
    w2 = np.outer(wq, wq) * prob.hx * prob.hy
    xe = prob.x0 + np.arange(prob.nx) * prob.Hx
    ye = prob.y0 + np.arange(prob.ny) * prob.Hy
    xq = xe[None, :, None, None] + tq[None, None, None, :] * prob.hx
    yq = ye[:, None, None, None] + tq[None, None, :, None] * prob.hy
    uh = np.einsum("rj,qi,abji->abrq", B, B, U, optimize=True)
    ux = np.einsum("rj,qi,abji->abrq", B, dB, U, optimize=True) / prob.hx
    uy = np.einsum("rj,qi,abji->abrq", dB, B, U, optimize=True) / prob.hy
    vh = np.einsum("rj,qi,abji->abrq", B, B, V, optimize=True)
    c, s = np.cos(OMEGA * t), np.sin(OMEGA * t)
    sx, sy = np.sin(K * xq), np.sin(K * yq)
    cx, cy = np.cos(K * xq), np.cos(K * yq)
    eu = uh - c * sx * sy
    ex = ux - c * K * cx * sy
    ey = uy - c * K * sx * cy
    ev = vh + OMEGA * s * sx * sy
    l2 = np.sqrt(np.sum(eu ** 2 * w2))
    en = np.sqrt(np.sum((ex ** 2 + ey ** 2 + ev ** 2) * w2))
    return float(l2), float(en)


def _run(n, N, p, flux):
    prob = dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux=flux, bc=BCS["dirichlet"])
    X, Y = dg2d.node_coords(prob)
    U0 = np.sin(K * X) * np.sin(K * Y)
    steps = int(np.ceil(T_FINAL / (CFL * prob.hx)))
    Ug, Vg, _, _ = _gpu(prob, U0, np.zeros_like(U0), T_FINAL / steps, steps)
    return prob.hx, _errors(Ug, Vg, prob, T_FINAL)


@pytest.mark.parametrize("flux", ["upwind", "central"])
@pytest.mark.parametrize("p", [3, 5, 7])
@pytest.mark.parametrize("table", ["Nfixed", "nfixed"])
def test_paper_dirichlet_rates(table, p, flux):
    r_l2, r_en = _golden()[(table, flux, p)]
    hs, e2, ee = [], [], []
    for n, N in GRIDS[table]:
        if N < p:
            continue
        h, (a, b) = _run(n, N, p, flux)
        hs.append(h)
        e2.append(a)
        ee.append(b)
    lh = np.log(hs)
    got_l2 = np.polyfit(lh, np.log(e2), 1)[0]
    got_en = np.polyfit(lh, np.log(ee), 1)[0]
    _say("%s %s p=%d: L2 rate %.2f (paper %.2f), energy rate %.2f (paper %.2f), L2 %s"
         % (table, flux, p, got_l2, r_l2, got_en, r_en, ["%.1e" % e for e in e2]))
    assert abs(got_en - r_en) <= 0.25
    if p in (3, 5):
        assert abs(got_l2 - r_l2) <= 0.6


# ---- walls on the PCG path (mapped elements, variable c^2) ----------------------------
def _pcg_gpu(n, N, p, Xm, Ym, c2, U0, V0, dt, steps, bc, flux="upwind", rtol=1e-13,
             precision="fp64"):
    from paper_2105_01722_amd import gdw
    s = gdw.Solver(n, n, N, p, flux=flux, xi=1.0, solver="pcg", coeff_variable=True,
                   mapped=True, pcg_rtol=rtol, precision=precision, bc=bc)
    try:
        s.set_coeff(c2, Xm, Ym)
        s.set_state(U0, V0)
        s.run(dt, steps)
        U, V = s.get_state()
        E = s.energy()
        st = s.stats(check=False)
    finally:
        s.close()
    return U.cpu().numpy(), V.cpu().numpy(), E, st


@pytest.mark.parametrize("bcname", ["dirichlet", "mixed", "x_periodic"])
@pytest.mark.parametrize("n,N,p,flux", [(3, 12, 5, "upwind"), (3, 8, 3, "central"),
                                        (2, 16, 5, "upwind"), (3, 7, 5, "upwind")])
def test_pcg_walls_match_dense_oracle(bcname, n, N, p, flux):
    """Curved mesh (straight outer sides) with variable c^2: the GPU PCG path with walls
    against the dense-direct general oracle with the same walls; register-operator
    kernels (N + 1 = 13, 9, 17) and the row layout (N = 7)."""
    _say("case: pcg walls", bcname, n, N, p, flux)
    X, Y = inputs.node_coords(n, n, N)
    Xm, Ym = inputs.mapped_coords(X, Y)
    c2 = inputs.c2_field(3, X, Y)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=4), Xm, Ym)
    V0 = 0.2 * inputs.fourier_field(inputs.fourier_modes(4, kmax=4), Xm, Ym)
    dt, steps = 0.1 / (n * N), 3
    Ug, Vg, Eg, st = _pcg_gpu(n, N, p, Xm, Ym, c2, U0, V0, dt, steps, BCS[bcname], flux=flux)
    assert st["status"] == 0 and st["fail_elem"] == -1
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux=flux, bc=BCS[bcname]),
                         Xm, Ym, c2)
    Uo, Vo = general.run(U0, V0, ops, dt, steps)
    assert_close(Ug, Uo, 1e-12)
    assert_close(Vg, Vo, 1e-12)
    Eo = general.energy(Uo, Vo, ops)
    assert abs(Eg - Eo) <= 1e-12 * abs(Eo)


def test_pcg_walls_cartesian_equal_fdm_walls():
    """Constant c^2 on a Cartesian grid: the PCG path with walls and the FDM path with
    the same walls give the same state (two GPU solvers, one scheme)."""
    _say("case: pcg walls vs fdm walls")
    n, N, p = 3, 12, 5
    prob = dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux="upwind", bc=BCS["mixed"])
    X, Y = dg2d.node_coords(prob)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=4), X, Y)
    V0 = np.zeros_like(U0)
    dt = 0.1 * prob.hx
    Uf, Vf, _, _ = _gpu(prob, U0, V0, dt, 4)
    Up, Vp, _, st = _pcg_gpu(n, N, p, X, Y, np.ones_like(X), U0, V0, dt, 4, BCS["mixed"])
    assert st["status"] == 0
    assert_close(Up, Uf, 1e-12)
    assert_close(Vp, Vf, 1e-12)


def test_pcg_walls_mixed_precision():
    """Mixed-precision PCG (FP32 inner iterations, FP64 refinement) with walls, against
    the dense oracle at the mixed path's bar (1e-10, as in test_gpu_pcg.py)."""
    _say("case: pcg walls mixed")
    n, N, p = 3, 12, 5
    X, Y = inputs.node_coords(n, n, N)
    Xm, Ym = inputs.mapped_coords(X, Y)
    c2 = inputs.c2_field(3, X, Y)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=4), Xm, Ym)
    V0 = 0.2 * inputs.fourier_field(inputs.fourier_modes(4, kmax=4), Xm, Ym)
    dt, steps = 0.1 / (n * N), 3
    bc = BCS["mixed"]
    Ug, Vg, _, st = _pcg_gpu(n, N, p, Xm, Ym, c2, U0, V0, dt, steps, bc, precision="mixed")
    assert st["status"] == 0 and st["mean_refine"] >= 1.0
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="upwind", bc=bc),
                         Xm, Ym, c2)
    Uo, Vo = general.run(U0, V0, ops, dt, steps)
    assert_close(Ug, Uo, 1e-10)
    assert_close(Vg, Vo, 1e-10)