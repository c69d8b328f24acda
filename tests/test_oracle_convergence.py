"""Pin of the constant-coefficient oracle against the convergence rates the paper prints
for its one-dimensional periodic experiment (Sec. 6, the two rate tables of "Periodic
Boundary Conditions in One Dimension"; values in tests/golden/rates_1d_periodic.txt).

The 2D oracle is run on a strip of nx elements by one element in y with y-independent
data.  Such states form an invariant subspace of the 2D scheme: the y-derivative traces
vanish, the N/S jumps are zero, S_y 1 = 0 and the mean equation reduces to the 1D one
(kappa / |Omega| w w^T with w = M_y 1 (x) M_x 1 acts as kappa / H_x on the x factor), so the
2D oracle restricted to it is the 1D method of the paper.  The test checks that invariance
and then evolves the travelling wave u = sin(8 pi (x - t)) with the paper's time step and
final time.

Two pieces of arithmetic replace the time loop, both exact rewrites of what the oracle
does: the restricted right-hand side is linear, so it is assembled column by column from
oracle calls; and N classical RK4 steps of a linear system are the N-th power of the
degree-4 Taylor polynomial of dt L (pinned separately in test_oracle_dg2d.py), taken by
repeated squaring.

Bars.  The energy-norm rates agree with the printed ones within 0.25 for every degree
and both fluxes.  The L2 rates depend more on the range of h used for the regression,
which the paper gives only in a figure; they are held to 0.6 for p = 3 and 5.  Not
compared: the L2 rate at p = 1 (the paper reports order reduction there, erratic in the
range) and at p = 7 for the upwind flux, where the L2 error of u stops falling at about
1e-9 in this range: that value moves by a factor of two when the assembled operator is
perturbed at the 1e-14 level (a rounding floor of the non-normal semi-discrete operator,
not a discretisation error), while the paper reports its p = 7 data down to 1e-13.
"""
import os

import numpy as np
import pytest

from oracle import dg2d, gd1d

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rates_1d_periodic.txt")
K_WAVE = 8.0 * np.pi
T_FINAL = 1.075
CFL = 0.075 / (2.0 * np.pi)


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


def _colours(n):
    """Smallest k >= 3 dividing n: elements e and e + k never share a neighbour, also
    across the periodic wrap, so one oracle call probes n / k elements at once."""
    for k in range(3, n + 1):
        if n % k == 0:
            return k
    return n


def _strip_operator(prob, ops):
    """The oracle's right-hand side restricted to y-independent states, as a dense matrix
    on z = (u, v), u and v each [nx][N+1] (the x-nodal values)."""
    n, n1 = prob.nx, prob.N + 1
    m = n * n1
    L = np.zeros((2 * m, 2 * m))
    k = _colours(n)
    worst = 0.0
    for c in range(k):
        owners = np.arange(c, n, k)
        for j in range(2 * n1):
            u = np.zeros((n, n1))
            v = np.zeros((n, n1))
            (u if j < n1 else v)[owners, j % n1] = 1.0
            U = np.broadcast_to(u[None, :, None, :], (1, n, n1, n1)).copy()
            V = np.broadcast_to(v[None, :, None, :], (1, n, n1, n1)).copy()
            du, dv = dg2d.rhs(U, V, ops)
            scale = max(np.abs(du).max(), np.abs(dv).max())
            worst = max(worst, np.abs(du - du[:, :, :1, :]).max() / scale,
                        np.abs(dv - dv[:, :, :1, :]).max() / scale)
            for e in owners:
                col = (j // n1) * m + e * n1 + j % n1
                for e2 in ((e - 1) % n, e, (e + 1) % n):
                    L[e2 * n1:(e2 + 1) * n1, col] = du[0, e2, 0, :]
                    L[m + e2 * n1:m + (e2 + 1) * n1, col] = dv[0, e2, 0, :]
    return L, worst


def _rk4_power(L, dt, steps):
    A = dt * L
    eye = np.eye(L.shape[0])
    P = eye + A @ (eye + A @ (eye + A @ (eye + A / 4.0) / 3.0) / 2.0)
    R = eye.copy()
    while steps:
        if steps & 1:
            R = R @ P
        P = P @ P
        steps >>= 1
    return R


def _errors(z, prob, t):
    """L2 error of u and energy-norm error (||u_x - u_h,x||^2 + ||v - v_h||^2)^(1/2) at
    time t, by (p+3)-point Gauss-Legendre quadrature per cell of the GD interpolants."""
    n, N, p = prob.nx, prob.N, prob.p
    n1 = N + 1
    m = n * n1
    u = z[:m].reshape(n, n1)
    v = z[m:].reshape(n, n1)
    xg, wg = gd1d.gauss_legendre(p + 3)
    tq = (np.arange(N)[:, None] + xg[None, :]).ravel()
    wq = np.tile(wg, N) * prob.hx
    B, dB = gd1d.basis_eval(N, p, tq)
    x = np.arange(n)[:, None] * prob.Hx + tq[None, :] * prob.hx
    ph = K_WAVE * (x - t)
    eu = u @ B.T - np.sin(ph)
    ev = v @ B.T + K_WAVE * np.cos(ph)
    ex = u @ dB.T / prob.hx - K_WAVE * np.cos(ph)
    return (float(np.sqrt(np.sum(eu ** 2 * wq))),
            float(np.sqrt(np.sum((ex ** 2 + ev ** 2) * wq))))


def _run(n, N, p, flux):
    prob = dg2d.CartProblem(nx=n, ny=1, N=N, p=p, flux=flux)
    ops = dg2d.CartOps(prob)
    L, worst = _strip_operator(prob, ops)
    assert worst < 1e-10, "y-independent states are not invariant (%.1e)" % worst
    steps = int(np.ceil(T_FINAL / (CFL * prob.hx)))
    x = (np.arange(n)[:, None] * prob.Hx + np.arange(N + 1)[None, :] * prob.hx).ravel()
    z0 = np.concatenate([np.sin(K_WAVE * x), -K_WAVE * np.cos(K_WAVE * x)])
    z = _rk4_power(L, T_FINAL / steps, steps) @ z0
    return prob.hx, _errors(z, prob, T_FINAL)


def _rates(grid, p, flux):
    hs, e2, ee = [], [], []
    for n, N in grid:
        h, (a, b) = _run(n, N, p, flux)
        hs.append(h)
        e2.append(a)
        ee.append(b)
    lh = np.log(hs)
    return np.polyfit(lh, np.log(e2), 1)[0], np.polyfit(lh, np.log(ee), 1)[0], e2


GRIDS = {
    "Nfixed": [(n, 10) for n in (8, 10, 12, 16, 20, 24, 32)],
    "nfixed": [(10, N) for N in (10, 12, 14, 16, 20, 24)],
}


@pytest.mark.parametrize("flux", ["upwind", "central"])
@pytest.mark.parametrize("p", [1, 3, 5, 7])
@pytest.mark.parametrize("table", ["Nfixed", "nfixed"])
def test_1d_periodic_rates_match_printed_table(table, p, flux):
    r_l2, r_en = _golden()[(table, flux, p)]
    grid = [(n, N) for n, N in GRIDS[table] if N >= p]
    got_l2, got_en, e2 = _rates(grid, p, flux)
    print("%s %s p=%d: L2 rate %.2f (paper %.2f), energy rate %.2f (paper %.2f), L2 errors %s"
          % (table, flux, p, got_l2, r_l2, got_en, r_en, ["%.1e" % e for e in e2]))
    assert abs(got_en - r_en) <= 0.25
    if p in (3, 5) or (p == 7 and flux == "central"):
        assert abs(got_l2 - r_l2) <= 0.6


def test_strip_reduction_is_the_1d_method():
    """The restricted operator is the same as the 1D scheme written directly from DG1,
    DG1_extra, DG2 and the fluxes of Sec. 2.2.1 with the 1D tables (one element column):
    y = S_hat^-1 F_u with S_hat = S + (1/H) w w^T, w = M 1; M v_t = -S u + F_v."""
    n, N, p = 5, 7, 3
    for flux in ("upwind", "central"):
        prob = dg2d.CartProblem(nx=n, ny=1, N=N, p=p, flux=flux)
        ops = dg2d.CartOps(prob)
        L, _ = _strip_operator(prob, ops)
        M, S, dL, dR = gd1d.element_1d(N, p, prob.Hx)
        al, be, ta = dg2d.flux_params(flux)
        w = M @ np.ones(N + 1)
        Sh = S + np.outer(w, w) / prob.Hx
        n1, m = N + 1, n * (N + 1)
        rng = np.random.default_rng(3)
        z = rng.standard_normal(2 * m)
        u = z[:m].reshape(n, n1)
        v = z[m:].reshape(n, n1)
        aE, aW = u @ dR, -(u @ dL)                  # outward normal derivatives
        vE, vW = v[:, -1], v[:, 0]
        aEn, vEn = np.roll(aW, -1), np.roll(vW, -1)  # east neighbour's west face
        aWn, vWn = np.roll(aE, 1), np.roll(vE, 1)
        suE = (1 - al) * (vEn - vE) - be * (aE + aEn)
        suW = (1 - al) * (vWn - vW) - be * (aW + aWn)
        svE = (1 - al) * aE - al * aEn + ta * (vEn - vE)
        svW = (1 - al) * aW - al * aWn + ta * (vWn - vW)
        Fu = np.outer(suE, dR) - np.outer(suW, dL)
        Fv = np.zeros_like(v)
        Fv[:, -1] += svE
        Fv[:, 0] += svW
        du = v + np.linalg.solve(Sh, Fu.T).T
        dv = np.linalg.solve(M, (Fv - u @ S.T).T).T
        want = np.concatenate([du.ravel(), dv.ravel()])
        got = L @ z
        assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
