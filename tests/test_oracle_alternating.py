"""Pins of the oracle's alternating flux (Sec. 2.2.1: alpha = 1, beta = tau = 0).

The printed flux takes superscript 1 as the inside of the element, which read literally
makes v* the element's own v on both sides of a face (two-valued).  The oracle fixes one
orientation per face (oracle/dg2d.py, face_alpha): v* from the element on the
low-coordinate side, (grad u)* from the element on the high side; alpha = 1/2 on wall
faces.  Pinned here by:

  * single-valuedness: across every interior face the two elements see the same v* and
    opposite n . (grad u)*, which the literal reading fails;
  * energy conservation (beta = tau = 0): dE/dt = 0 on Cartesian and curved variable-c^2
    meshes, periodic and with walls;
  * the affine-mesh reduction of the general (quadrature) oracle to the Cartesian one;
  * the convergence rates printed in the paper's 1D periodic tables (A.-flux columns,
    tests/golden/rates_1d_periodic.txt): the energy-norm rate of the alternating flux is
    the suboptimal p - 1 with N + 1 = 11 fixed and about p - 1/2 with n = 10 fixed, a
    signature no other orientation or alpha gives.
"""
import os

import numpy as np
import pytest

from oracle import dg2d, general
from paper_2105_01722_amd import inputs

import test_oracle_convergence as conv


def _state(prob, seed):
    rng = np.random.default_rng(seed)
    shp = (prob.ny, prob.nx, prob.N + 1, prob.N + 1)
    return rng.standard_normal(shp), rng.standard_normal(shp)


def _sigmas(prob, ops, U, V, alpha_of):
    tr = dg2d.traces(U, V, ops)
    nb = dg2d.neighbour_traces(tr, prob.bc)
    return tr, {f: dg2d.face_sigmas(tr[f][0], tr[f][1], nb[f][0], nb[f][1], alpha_of(f), 0.0, 0.0)
                for f in "EWNS"}


def test_alternating_flux_is_single_valued():
    prob = dg2d.CartProblem(nx=3, ny=2, N=6, p=3, flux="alternating")
    ops = dg2d.CartOps(prob)
    U, V = _state(prob, 1)
    for alpha_of, ok in ((lambda f: dg2d.face_alphas(prob, f)[:, :, None], True),
                         (lambda f: 1.0, False)):
        tr, sig = _sigmas(prob, ops, U, V, alpha_of)
        # x faces: E of (ey, ex) against W of (ey, ex + 1); y faces: N of (ey, ex) against S
        vE = tr["E"][1] + sig["E"][0]
        vW = np.roll(tr["W"][1] + sig["W"][0], -1, axis=1)
        gE, gW = sig["E"][1], np.roll(sig["W"][1], -1, axis=1)
        vN = tr["N"][1] + sig["N"][0]
        vS = np.roll(tr["S"][1] + sig["S"][0], -1, axis=0)
        gN, gS = sig["N"][1], np.roll(sig["S"][1], -1, axis=0)
        err = max(np.abs(vE - vW).max(), np.abs(gE + gW).max(), np.abs(vN - vS).max(),
                  np.abs(gN + gS).max())
        if ok:
            assert err <= 1e-12
        else:
            assert err > 1e-2
    # on the oriented faces v* is the low side's value and (grad u)* the high side's
    tr, sig = _sigmas(prob, ops, U, V, lambda f: dg2d.face_alphas(prob, f)[:, :, None])
    np.testing.assert_allclose(tr["E"][1] + sig["E"][0], tr["E"][1], atol=1e-13)
    np.testing.assert_allclose(sig["E"][1], -np.roll(tr["W"][0], -1, axis=1), atol=1e-12)


@pytest.mark.parametrize("bc", [("periodic",) * 4, ("dirichlet",) * 4,
                                ("neumann", "neumann", "dirichlet", "dirichlet")])
@pytest.mark.parametrize("N,p", [(6, 3), (7, 5)])
def test_alternating_conserves_energy_cartesian(N, p, bc):
    """d/dt [1/2 V^T M V + 1/2 c^2 U^T S U] = V^T M dV + c^2 U^T S dU = 0 for the full
    right-hand side (solves included), with walls where given."""
    prob = dg2d.CartProblem(nx=3, ny=3, N=N, p=p, flux="alternating", c2=1.3, bc=bc)
    ops = dg2d.CartOps(prob)
    U, V = _state(prob, 2)
    dU, dV = dg2d.rhs(U, V, ops)
    n = prob.nx * prob.ny
    u, v = U.reshape(n, -1), V.reshape(n, -1)
    rate = (np.einsum("ei,ij,ej->", v, ops.M2, dV.reshape(n, -1))
            + prob.c2 * np.einsum("ei,ij,ej->", u, ops.S2, dU.reshape(n, -1)))
    scale = np.abs(np.einsum("ei,ij,ej->e", v, ops.M2, dV.reshape(n, -1))).sum()
    assert abs(rate) < 1e-12 * scale
    assert abs(dg2d.energy_rate(U, V, ops)) < 1e-12 * scale


@pytest.mark.parametrize("bc", [("periodic",) * 4, ("dirichlet", "dirichlet", "neumann", "neumann")])
def test_alternating_conserves_energy_curved_variable(bc):
    n, N, p = 3, 6, 3
    X, Y = inputs.node_coords(n, n, N)
    Xm, Ym = inputs.mapped_coords(X, Y)
    c2 = inputs.c2_field(3, X, Y)
    rng = np.random.default_rng(4)
    U, V = rng.standard_normal(X.shape), rng.standard_normal(X.shape)
    g = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="alternating", bc=bc),
                       Xm, Ym, c2)
    dU, dV = general.rhs(U, V, g)
    ne = n * n
    rate = (np.einsum("ei,eij,ej->", V.reshape(ne, -1), g.M, dV.reshape(ne, -1))
            + np.einsum("ei,eij,ej->", U.reshape(ne, -1), g.S, dU.reshape(ne, -1)))
    scale = np.abs(np.einsum("ei,eij,ej->e", V.reshape(ne, -1), g.M, dV.reshape(ne, -1))).sum()
    assert abs(rate) < 1e-11 * scale


@pytest.mark.parametrize("bc", [("periodic",) * 4, ("dirichlet",) * 4])
def test_general_alternating_on_affine_mesh_equals_cartesian(bc):
    n, N, p, c2 = 3, 6, 3, 1.7
    X, Y = inputs.node_coords(n, n, N, Lx=1.3, Ly=0.7, x0=-0.2, y0=0.1)
    g = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="alternating", bc=bc),
                       X, Y, np.full_like(X, c2))
    c = dg2d.CartOps(dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux="alternating", c2=c2,
                                      Lx=1.3, Ly=0.7, x0=-0.2, y0=0.1, bc=bc))
    rng = np.random.default_rng(2)
    U, V = rng.standard_normal(X.shape), rng.standard_normal(X.shape)
    for x, y in zip(general.rhs(U, V, g), dg2d.rhs(U, V, c)):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(y).max()


def test_alternating_spectrum_stable_at_bench_cfl():
    """The dense semi-discrete operator of a 2 x 2 periodic instance (N = 8, p = 3) has a
    purely imaginary spectrum (energy conserving), and RK4 is stable at dt = 0.3 h."""
    prob = dg2d.CartProblem(nx=2, ny=2, N=8, p=3, flux="alternating")
    ops = dg2d.CartOps(prob)
    m = prob.nx * prob.ny * (prob.N + 1) ** 2
    L = np.zeros((2 * m, 2 * m))
    for j in range(2 * m):
        z = np.zeros(2 * m)
        z[j] = 1.0
        U = z[:m].reshape(prob.ny, prob.nx, prob.N + 1, prob.N + 1)
        V = z[m:].reshape(U.shape)
        dU, dV = dg2d.rhs(U, V, ops)
        L[:, j] = np.concatenate([dU.ravel(), dV.ravel()])
    lam = np.linalg.eigvals(L)
    rho = np.abs(lam).max()
    assert np.abs(lam.real).max() <= 1e-9 * rho
    z = 0.3 * prob.hx * lam
    R4 = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    assert np.abs(R4).max() <= 1.0 + 1e-12


# ---- the paper's 1D periodic A.-flux rates --------------------------------------------
# The regressions' ranges of h appear only in the paper's figures.  With N + 1 = 11 fixed
# the range n = 10 ... 40 (the text mentions regressing its p = 7 data over the first 31
# points) reproduces the printed A.-flux rates to 0.07 (every n or every second n, as
# here, give the same rates); the 7-grid range of the U./C. pins (conv.GRIDS) leaves the
# alternating energy rates 0.4-0.5 short at p = 5, 7.
GRIDS_ALT = {"Nfixed": [(n, 10) for n in range(10, 41, 2)], "nfixed": conv.GRIDS["nfixed"]}


@pytest.mark.parametrize("p", [1, 3, 5, 7])
@pytest.mark.parametrize("table", ["Nfixed", "nfixed"])
def test_1d_periodic_alternating_rates_match_printed_table(table, p):
    r_l2, r_en = conv._golden()[(table, "alternating", p)]
    grid = [(n, N) for n, N in GRIDS_ALT[table] if N >= p]
    got_l2, got_en, e2 = conv._rates(grid, p, "alternating")
    print("%s alternating p=%d: L2 rate %.2f (paper %.2f), energy rate %.2f (paper %.2f)"
          % (table, p, got_l2, r_l2, got_en, r_en))
    assert abs(got_en - r_en) <= 0.25
    if p in (3, 5):
        assert abs(got_l2 - r_l2) <= 0.6
