"""GPU parity of the alternating flux (Sec. 2.2.1, alpha = 1 with the face orientation of
include/gdw.h: v* from the element on the low-coordinate side, (grad u)* from the one on
the high side; alpha = 1/2 on wall faces) against the FP64 oracle, through the C ABI, on
the constant-coefficient path (FP64 and FP32 storage, periodic and walls) and on the PCG
path (curved mesh, variable c^2; register-operator and row-layout kernels), and the
paper's 2D Dirichlet rates for the alternating flux (A.-flux columns of
tests/golden/rates_2d_dirichlet.txt).

Bars as for the other fluxes: FP64 relative l2 <= 1e-12 against the oracle (max <= 1e-11),
FP32 storage <= 1e-6; energy-norm rates within 0.25 of the printed ones and L2 rates
within 0.6 for p = 3 and 5.
"""
import sys

import numpy as np
import pytest

from oracle import dg2d, general
from paper_2105_01722_amd import inputs

from _cmp import assert_close, rel as _rel, relmax as _relmax  # noqa: E402

pytestmark = pytest.mark.gpu

BCS = {"periodic": ("periodic",) * 4, "dirichlet": ("dirichlet",) * 4,
       "mixed": ("dirichlet", "dirichlet", "neumann", "neumann")}


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _fdm(prob, U0, V0, dt, steps, precision="fp64"):
    from paper_2105_01722_amd import gdw
    s = gdw.Solver(prob.nx, prob.ny, prob.N, prob.p, c2=prob.c2, flux=prob.flux,
                   precision=precision, Lx=prob.Lx, Ly=prob.Ly, x0=prob.x0, y0=prob.y0,
                   bc=prob.bc)
    try:
        s.set_state(U0, V0)
        E0 = s.energy()
        s.run(dt, steps)
        U, V = s.get_state()
        E = s.energy()
        assert s.stats()["status"] == 0
    finally:
        s.close()
    return U.cpu().numpy(), V.cpu().numpy(), E0, E


@pytest.mark.parametrize("n,N,p,bc,precision", [
    (3, 16, 5, "periodic", "fp64"), (5, 8, 3, "periodic", "fp64"), (2, 12, 7, "periodic", "fp64"),
    (5, 8, 3, "dirichlet", "fp64"), (3, 16, 5, "mixed", "fp64"), (4, 10, 5, "periodic", "fp64"),
    (3, 16, 5, "periodic", "fp32"), (5, 8, 3, "mixed", "fp32")])
def test_fdm_alternating_matches_oracle(n, N, p, bc, precision):
    _say("case: fdm alternating", n, N, p, bc, precision)
    prob = dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux="alternating", bc=BCS[bc], c2=1.2)
    X, Y = dg2d.node_coords(prob)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=4), X, Y)
    V0 = 0.3 * inputs.fourier_field(inputs.fourier_modes(3, kmax=4), X, Y)
    if bc != "periodic":
        U0 = U0 * np.sin(np.pi * X) * np.sin(np.pi * Y)
        V0 = V0 * np.sin(np.pi * X) * np.sin(np.pi * Y)
    dt, steps = 0.1 * prob.hx, 6
    Ug, Vg, E0, Eg = _fdm(prob, U0, V0, dt, steps, precision)
    ops = dg2d.CartOps(prob)
    Uo, Vo = dg2d.run(U0, V0, ops, dt, steps)
    _say("  rel l2 U %.2e V %.2e, max U %.2e V %.2e" % (_rel(Ug, Uo), _rel(Vg, Vo),
                                                       _relmax(Ug, Uo), _relmax(Vg, Vo)))
    bar = 1e-12 if precision == "fp64" else 1e-6
    assert_close(Ug, Uo, bar)
    assert_close(Vg, Vo, bar)
    Eo = dg2d.energy(Uo, Vo, ops)
    assert abs(Eg - Eo) <= (1e-12 if precision == "fp64" else 1e-6) * abs(Eo)
    assert abs(Eg - E0) <= 1e-6 * E0            # conservative flux: RK4 drift only


@pytest.mark.parametrize("n,N,p,bc", [(3, 12, 5, "periodic"), (3, 12, 5, "mixed"),
                                      (3, 8, 3, "dirichlet"), (3, 7, 5, "periodic"),
                                      (2, 16, 5, "periodic")])
def test_pcg_alternating_matches_dense_oracle(n, N, p, bc):
    """Curved mesh (straight outer sides), variable c^2, PCG at rtol 1e-13 against the
    dense-direct general oracle: register kernels (N + 1 = 13, 9, 17) and the row layout
    (N = 7)."""
    from paper_2105_01722_amd import gdw
    _say("case: pcg alternating", n, N, p, bc)
    X, Y = inputs.node_coords(n, n, N)
    Xm, Ym = inputs.mapped_coords(X, Y)
    c2 = inputs.c2_field(3, X, Y)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=3), Xm, Ym)
    V0 = 0.3 * inputs.fourier_field(inputs.fourier_modes(3, kmax=3), Xm, Ym)
    dt, steps = 0.05 / (n * N), 3
    s = gdw.Solver(n, n, N, p, flux="alternating", solver="pcg", coeff_variable=True,
                   mapped=True, pcg_rtol=1e-13, bc=BCS[bc])
    try:
        s.set_coeff(c2, Xm, Ym)
        s.set_state(U0, V0)
        s.run(dt, steps)
        Ug, Vg = (x.cpu().numpy() for x in s.get_state())
        Eg = s.energy()
        assert s.stats()["status"] == 0
    finally:
        s.close()
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="alternating",
                                            bc=BCS[bc]), Xm, Ym, c2)
    Uo, Vo = general.run(U0, V0, ops, dt, steps)
    _say("  rel l2 U %.2e V %.2e, max U %.2e V %.2e" % (_rel(Ug, Uo), _rel(Vg, Vo),
                                                       _relmax(Ug, Uo), _relmax(Vg, Vo)))
    assert_close(Ug, Uo, 1e-12)
    assert_close(Vg, Vo, 1e-12)
    Eo = general.energy(Uo, Vo, ops)
    assert abs(Eg - Eo) <= 1e-12 * abs(Eo)


# ---- the paper's 2D Dirichlet experiment with the alternating flux -----------------------
# The paper regresses its alternating-flux data with N + 1 = 11 fixed over "the 25
# coarsest grids" of its (unprinted) range; n = 10 ... 34 is taken here.
ALT_GRIDS = {"Nfixed": [(n, 10) for n in range(10, 35)],
             "nfixed": [(10, N) for N in (10, 12, 14, 16, 20, 24)]}


@pytest.mark.parametrize("p", [3, 5, 7])
@pytest.mark.parametrize("table", ["Nfixed", "nfixed"])
def test_paper_dirichlet_rates_alternating(table, p):
    import test_gpu_walls as tw
    r_l2, r_en = tw._golden()[(table, "alternating", p)]
    hs, e2, ee = [], [], []
    for n, N in ALT_GRIDS[table]:
        if N < p:
            continue
        h, (a, b) = tw._run(n, N, p, "alternating")
        hs.append(h)
        e2.append(a)
        ee.append(b)
    lh = np.log(hs)
    got_l2 = np.polyfit(lh, np.log(e2), 1)[0]
    got_en = np.polyfit(lh, np.log(ee), 1)[0]
    _say("%s alternating p=%d: L2 rate %.2f (paper %.2f), energy rate %.2f (paper %.2f), L2 %s"
         % (table, p, got_l2, r_l2, got_en, r_en, ["%.1e" % e for e in e2]))
    assert abs(got_en - r_en) <= 0.25
    if p in (3, 5):
        assert abs(got_l2 - r_l2) <= 0.6
