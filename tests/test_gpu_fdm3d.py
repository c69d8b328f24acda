"""GPU parity of the 3D box-element path (Sec. 2.2 with d = 3) against the 3D oracle,
through the C ABI.

Bars as in 2D: FP64 relative l2 <= 1e-12 against the oracle (max <= 1e-11), FP32 storage
<= 1e-6; energy within 1e-12 (FP64).  Grids span several 2-element workgroup tiles with a
ragged last tile, the specialised kernels (N + 1 = 9, 10) and the generic one, the three
fluxes and walls on all three axes.  The full-size case runs the benchmark's 3D grid in
the launch configuration bench.py times and compares sampled elements with the oracle on
periodic patches of (8 s + 1)^3 elements (an element's state after s steps depends only
on elements within Manhattan distance 4 s).
"""
import sys

import numpy as np
import pytest

from oracle import dg3d
from paper_2105_01722_amd import inputs

from _cmp import assert_close, rel as _rel, relmax as _relmax  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu(prob, U0, V0, dt, steps, precision="fp64"):
    from paper_2105_01722_amd import gdw
    s = gdw.Solver(prob.nx, prob.ny, prob.N, prob.p, nz=prob.nz, c2=prob.c2, flux=prob.flux,
                   xi=prob.xi, precision=precision, Lx=prob.Lx, Ly=prob.Ly, Lz=prob.Lz,
                   x0=prob.x0, y0=prob.y0, z0=prob.z0, bc=prob.bc[:4], bcz=prob.bc[4:])
    try:
        s.set_state(U0, V0)
        s.run(dt, steps)
        U, V = s.get_state()
        E = s.energy()
        st = s.stats()
    finally:
        s.close()
    return U.cpu().numpy(), V.cpu().numpy(), E, st


WALLS = ("dirichlet", "dirichlet", "neumann", "neumann", "dirichlet", "dirichlet")


@pytest.mark.parametrize("n,N,p,flux,bc,precision", [
    ((3, 2, 2), 8, 3, "upwind", ("periodic",) * 6, "fp64"),
    ((2, 2, 3), 9, 5, "central", ("periodic",) * 6, "fp64"),
    ((2, 3, 2), 6, 3, "alternating", ("periodic",) * 6, "fp64"),
    ((3, 2, 2), 8, 3, "upwind", WALLS, "fp64"),
    ((2, 2, 2), 5, 5, "upwind", ("periodic",) * 6, "fp64"),
    ((3, 3, 1), 8, 3, "upwind", ("periodic",) * 6, "fp64"),
    ((3, 2, 2), 8, 3, "upwind", ("periodic",) * 6, "fp32"),
    ((2, 2, 3), 9, 5, "alternating", WALLS, "fp32"),
])
def test_3d_matches_oracle(n, N, p, flux, bc, precision):
    _say("case: 3d", n, N, p, flux, bc[0], bc[2], bc[4], precision)
    nx, ny, nz = n
    prob = dg3d.CartProblem3(nx=nx, ny=ny, nz=nz, N=N, p=p, Lx=1.0, Ly=0.9, Lz=1.1, c2=1.3,
                             flux=flux, xi=np.sqrt(1.3), bc=bc)
    X, Y, Z = dg3d.node_coords(prob)
    U0 = inputs.fourier_field3(inputs.fourier_modes3(2, kmax=2), X, Y, Z)
    V0 = 0.5 * inputs.fourier_field3(inputs.fourier_modes3(3, kmax=2), X, Y, Z)
    dt, steps = 0.08 * prob.h[0], 5
    Ug, Vg, Eg, st = _gpu(prob, U0, V0, dt, steps, precision)
    ops = dg3d.CartOps3(prob)
    Uo, Vo = dg3d.run(U0, V0, ops, dt, steps)
    _say("  rel l2 U %.2e V %.2e, max U %.2e V %.2e" % (_rel(Ug, Uo), _rel(Vg, Vo),
                                                       _relmax(Ug, Uo), _relmax(Vg, Vo)))
    bar = 1e-12 if precision == "fp64" else 1e-6
    assert_close(Ug, Uo, bar)
    assert_close(Vg, Vo, bar)
    Eo = dg3d.energy(Uo, Vo, ops)
    assert abs(Eg - Eo) <= (1e-12 if precision == "fp64" else 1e-6) * abs(Eo)
    assert st["steps_taken"] == steps and st["dof_updates"] == steps * nx * ny * nz * (N + 1) ** 3


def test_3d_standing_wave_and_energy():
    """u = sin 2 pi x sin 2 pi y sin 2 pi z cos(2 sqrt(3) pi t), central flux: close to the
    exact wave at t = 0.1 and the energy conserved up to the RK4 drift."""
    from paper_2105_01722_amd import gdw
    n, N, p = 4, 8, 3
    X, Y, Z = inputs.node_coords3(n, n, n, N)
    U0 = np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(2 * np.pi * Z)
    s = gdw.Solver(n, n, N, p, nz=n, flux="central")
    try:
        s.set_state(U0, np.zeros_like(U0))
        E0 = s.energy()
        T = 0.1
        steps = int(np.ceil(T / (0.2 / (n * N))))
        s.run(T / steps, steps)
        U, _ = s.get_state()
        E = s.energy()
    finally:
        s.close()
    exact = np.cos(2 * np.sqrt(3.0) * np.pi * T) * U0
    err = np.abs(U.cpu().numpy() - exact).max()
    _say("  standing wave max error %.2e, energy drift %.1e" % (err, abs(E - E0) / E0))
    assert err < 2e-4
    assert abs(E - E0) <= 1e-6 * E0


def _patch3(A, c, R):
    """Elements c +- R (periodic wrap) of A [nz, ny, nx, ...]."""
    idx = [np.arange(c[k] - R, c[k] + R + 1) % A.shape[k] for k in range(3)]
    return A[np.ix_(*idx)].copy()


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_3d_full_size_sampled(precision, bar):
    """The 3D benchmark grid (48^3 elements, N = 8, p = 3, upwind, dt = 0.12 h), 2 steps,
    sampled elements at a corner and inside against the oracle on 17^3-element patches."""
    import torch
    from paper_2105_01722_amd import gdw
    n, N, p, steps = 48, 8, 3, 2
    _say("case: 3d full size", precision)
    X, Y, Z = inputs.node_coords3(n, n, n, N)
    U0 = inputs.fourier_field3(inputs.fourier_modes3(2), X, Y, Z)
    V0 = 20.0 * inputs.fourier_field3(inputs.fourier_modes3(4), X, Y, Z)
    dt = 0.12 / (n * N)
    s = gdw.Solver(n, n, N, p, nz=n, flux="upwind", xi=1.0, precision=precision)
    try:
        s.set_state(torch.from_numpy(U0).cuda(), torch.from_numpy(V0).cuda())
        s.run(dt, steps)
        Ug, Vg = (x.cpu().numpy() for x in s.get_state())
        assert s.stats()["status"] == 0
    finally:
        s.close()
    R = 4 * steps
    P = 2 * R + 1
    prob = dg3d.CartProblem3(nx=P, ny=P, nz=P, N=N, p=p, Lx=P / n, Ly=P / n, Lz=P / n,
                             flux="upwind")
    ops = dg3d.CartOps3(prob)
    gu, gv, ru, rv = [], [], [], []
    for c in [(0, 0, 0), (n // 2, n // 3, n - 1), (n // 5, 3 * n // 4, n // 2)]:
        Uo, Vo = dg3d.run(_patch3(U0, c, R), _patch3(V0, c, R), ops, dt, steps)
        ru.append(Uo[R, R, R]); rv.append(Vo[R, R, R])
        gu.append(Ug[c]); gv.append(Vg[c])
    gu, gv, ru, rv = (np.array(x) for x in (gu, gv, ru, rv))
    _say("  sampled rel l2 U %.2e V %.2e, max U %.2e V %.2e" % (
        _rel(gu, ru), _rel(gv, rv), _relmax(gu, ru), _relmax(gv, rv)))
    assert_close(gu, ru, bar)
    assert_close(gv, rv, bar)
