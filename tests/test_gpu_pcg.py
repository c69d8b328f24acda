"""GPU parity of the variable-coefficient / mapped-element path (PCG element solves,
Sec. 7.1) against the FP64 oracle, through the C ABI.

Bars: with pcg_rtol = 1e-13 the GPU state after a few RK4 steps matches the oracle's
dense-direct run to relative l2 <= 1e-12 (the oracle's own PCG at the same tolerance
sits 1e-13 below that); with the Cartesian constant-coefficient special case the
preconditioner is exact (at most one iteration per solve); at pcg_rtol = 1e-10 the
GPU and oracle PCG iteration counts agree (mean within 3 %, max within 2).
"""
import sys

import numpy as np
import pytest

from oracle import dg2d, general, pcg
from paper_2105_01722_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


from _cmp import assert_close, rel as _rel, relmax as _relmax  # noqa: E402


def _problem(n, N, p, mapped, variable, seed=3, kmax=4):
    X, Y = inputs.node_coords(n, n, N)
    c2 = inputs.c2_field(seed, X, Y) if variable else np.full_like(X, 1.0)
    Xm, Ym = inputs.mapped_coords(X, Y) if mapped else (X, Y)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=kmax), Xm, Ym)
    V0 = 0.2 * inputs.fourier_field(inputs.fourier_modes(4, kmax=kmax), Xm, Ym)
    return Xm, Ym, c2, U0, V0


def _gpu(n, N, p, Xm, Ym, c2, U0, V0, dt, steps, mapped, variable, flux="upwind", rtol=1e-13,
         maxit=200, give_coords=True, precision="fp64"):
    from paper_2105_01722_amd import gdw
    s = gdw.Solver(n, n, N, p, flux=flux, xi=1.0, solver="pcg", coeff_variable=variable,
                   mapped=mapped, pcg_rtol=rtol, pcg_maxit=maxit, precision=precision)
    s.set_coeff(c2 if variable else None, Xm if (mapped or give_coords) else None,
                Ym if (mapped or give_coords) else None)
    s.set_state(U0, V0)
    s.run(dt, steps)
    U, V = s.get_state()
    E = s.energy()
    st = s.stats(check=False)
    s.close()
    return U.cpu().numpy(), V.cpu().numpy(), E, st


# Kernel families covered: row layout (N = 6, 7), the operator in registers for every
# compiled (N + 1, p) pair (9: p = 3, 5, 7; 13: p = 3, 5, 7; 17: p = 3, 5) and the streamed
# operator (17: p = 7, mapped and Cartesian).  N = 12, p = 7 also covers nodes that lie in
# more than 8 cell windows of the closure (lifts).
@pytest.mark.parametrize("n,N,p,mapped,variable", [(3, 6, 3, True, True), (3, 12, 5, True, True),
                                                   (3, 12, 5, False, True), (2, 8, 7, True, True),
                                                   (3, 7, 5, True, False), (2, 8, 3, True, True),
                                                   (2, 8, 5, True, True), (2, 12, 3, True, True),
                                                   (2, 12, 7, True, True), (2, 16, 3, True, True),
                                                   (2, 16, 5, True, True), (2, 16, 7, True, True),
                                                   (2, 16, 7, False, True)])
def test_pcg_matches_dense_oracle(n, N, p, mapped, variable):
    _say("case: pcg vs dense", n, N, p, mapped, variable)
    Xm, Ym, c2, U0, V0 = _problem(n, N, p, mapped, variable)
    dt, steps = 0.1 / (n * N), 3
    Ug, Vg, Eg, st = _gpu(n, N, p, Xm, Ym, c2, U0, V0, dt, steps, mapped, variable)
    assert st["status"] == 0 and st["fail_elem"] == -1
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="upwind"), Xm, Ym, c2)
    Uo, Vo = general.run(U0, V0, ops, dt, steps)
    assert_close(Ug, Uo, 1e-12)
    assert_close(Vg, Vo, 1e-12)
    Eo = general.energy(Uo, Vo, ops)
    assert abs(Eg - Eo) <= 1e-12 * abs(Eo)
    if not mapped:
        assert st["max_it_M"] <= 1


def test_pcg_cartesian_constant_equals_fdm_and_exact_preconditioner():
    """Constant c^2 on Cartesian elements through the PCG path: the preconditioner is
    the element matrix itself (at most one iteration) and the result is the FDM one."""
    _say("case: pcg cartesian constant")
    n, N, p = 3, 12, 5
    X, Y = inputs.node_coords(n, n, N)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=4), X, Y)
    V0 = np.zeros_like(U0)
    dt, steps = 0.1 / (n * N), 3
    Ug, Vg, _, st = _gpu(n, N, p, X, Y, None, U0, V0, dt, steps, mapped=False, variable=False,
                         give_coords=False)
    assert st["max_it_S"] <= 1 and st["max_it_M"] <= 1
    Uo, Vo = dg2d.run(U0, V0, dg2d.CartOps(dg2d.CartProblem(nx=n, ny=n, N=N, p=p, flux="upwind")),
                      dt, steps)
    assert_close(Ug, Uo, 1e-12)
    assert_close(Vg, Vo, 1e-12)


def test_pcg_iteration_counts_match_oracle():
    _say("case: pcg iteration counts")
    n, N, p = 3, 12, 5
    Xm, Ym, c2, U0, V0 = _problem(n, N, p, True, True)
    dt, steps = 0.1 / (n * N), 2
    _, _, _, st = _gpu(n, N, p, Xm, Ym, c2, U0, V0, dt, steps, True, True, rtol=1e-10)
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="upwind"), Xm, Ym, c2)
    f = pcg.PcgRhs(ops, rtol=1e-10)
    general.run(U0, V0, ops, dt, steps, f=f)
    itS, itM = np.array(f.its_S), np.array(f.its_M)
    assert st["solves"] == itS.size
    assert abs(st["mean_it_S"] - itS.mean()) <= 0.03 * itS.mean()
    assert abs(st["mean_it_M"] - itM.mean()) <= 0.03 * itM.mean()
    assert abs(st["max_it_S"] - itS.max()) <= 2 and abs(st["max_it_M"] - itM.max()) <= 2


def test_pcg_central_energy_conserved():
    """Central flux on a curved mesh with variable c^2: the semi-discrete energy is
    conserved, so over a few small steps it changes only by RK4's O(dt^5) damping."""
    _say("case: pcg central energy")
    n, N, p = 3, 8, 3
    Xm, Ym, c2, U0, V0 = _problem(n, N, p, True, True, kmax=2)
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="central"), Xm, Ym, c2)
    E0 = general.energy(U0, V0, ops)
    _, _, Eg, st = _gpu(n, N, p, Xm, Ym, c2, U0, V0, 0.02 / (n * N), 5, True, True, flux="central")
    assert st["status"] == 0
    assert abs(Eg - E0) <= 1e-9 * E0


def test_pcg_maxit_reports_enoconv():
    """A too small iteration limit is reported (ENOCONV, element id); kernels still finish."""
    _say("case: pcg maxit")
    from paper_2105_01722_amd import gdw
    n, N, p = 2, 8, 3
    Xm, Ym, c2, U0, V0 = _problem(n, N, p, True, True)
    _, _, _, st = _gpu(n, N, p, Xm, Ym, c2, U0, V0, 0.01, 1, True, True, rtol=1e-13, maxit=2)
    assert st["status"] == gdw.GDW_ENOCONV and 0 <= st["fail_elem"] < n * n


@pytest.mark.parametrize("n,N,p,mapped,variable", [(3, 12, 5, True, True), (3, 8, 3, True, True),
                                                   (2, 16, 3, False, True), (2, 8, 7, True, True)])
def test_pcg_mixed_matches_dense_oracle(n, N, p, mapped, variable):
    """Mixed precision (FP32 operator in the inner iterations, FP64 residual refinement with
    A = hi + lo): the refined solution meets the same FP64 residual tolerance with an
    operator represented to about 2^-48 (3.6e-15) instead of 2^-53, so the state is
    compared with the dense oracle at 1e-10 (the FP64 bar of 1e-12 times that ratio,
    with margin); at least one refinement sweep must have run."""
    _say("case: pcg mixed vs dense", n, N, p, mapped, variable)
    Xm, Ym, c2, U0, V0 = _problem(n, N, p, mapped, variable)
    dt, steps = 0.1 / (n * N), 3
    Ug, Vg, Eg, st = _gpu(n, N, p, Xm, Ym, c2, U0, V0, dt, steps, mapped, variable,
                          precision="mixed")
    assert st["status"] == 0
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="upwind"), Xm, Ym, c2)
    Uo, Vo = general.run(U0, V0, ops, dt, steps)
    eu, ev = _rel(Ug, Uo), _rel(Vg, Vo)
    _say("  rel U %.2e V %.2e  its S %.2f M %.2f refine %.2f"
         % (eu, ev, st["mean_it_S"], st["mean_it_M"], st["mean_refine"]))
    assert_close(Ug, Uo, 1e-10)
    assert_close(Vg, Vo, 1e-10)
    Eo = general.energy(Uo, Vo, ops)
    assert abs(Eg - Eo) <= 1e-10 * abs(Eo)
    assert st["mean_refine"] >= 1.0


@pytest.mark.parametrize("n,N,p,mapped,variable", [(3, 12, 5, True, True), (2, 8, 7, True, True),
                                                   (3, 12, 3, False, True), (2, 8, 5, True, True),
                                                   (2, 12, 7, True, True)])
def test_pcg_pc32_matches_dense_oracle(n, N, p, mapped, variable):
    """GDW_MIXED_PC32: the preconditioner's four transforms on the FP32 matrix cores inside
    the FP64 recurrence.  Operator products, residuals and the stop test stay FP64, so the
    solves meet the same rtol: the state meets the FP64 bar against the dense oracle
    (1e-12 at pcg_rtol 1e-13), and the iteration means stay within 0.5 of the FP64 run's
    (a preconditioner perturbed at 2^-24 changes the Krylov space only at that level)."""
    _say("case: pcg pc32 vs dense", n, N, p, mapped, variable)
    Xm, Ym, c2, U0, V0 = _problem(n, N, p, mapped, variable)
    dt, steps = 0.1 / (n * N), 3
    Ug, Vg, Eg, st = _gpu(n, N, p, Xm, Ym, c2, U0, V0, dt, steps, mapped, variable,
                          precision="pc32")
    _, _, _, sf = _gpu(n, N, p, Xm, Ym, c2, U0, V0, dt, steps, mapped, variable)
    assert st["status"] == 0 and st["fail_elem"] == -1
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="upwind"), Xm, Ym, c2)
    Uo, Vo = general.run(U0, V0, ops, dt, steps)
    _say("  rel U %.2e V %.2e  its S %.2f (fp64 %.2f) M %.2f (fp64 %.2f)"
         % (_rel(Ug, Uo), _rel(Vg, Vo), st["mean_it_S"], sf["mean_it_S"], st["mean_it_M"],
            sf["mean_it_M"]))
    assert_close(Ug, Uo, 1e-12)
    assert_close(Vg, Vo, 1e-12)
    Eo = general.energy(Uo, Vo, ops)
    assert abs(Eg - Eo) <= 1e-12 * abs(Eo)
    assert abs(st["mean_it_S"] - sf["mean_it_S"]) <= 0.5
    assert abs(st["mean_it_M"] - sf["mean_it_M"]) <= 0.5


def test_pcg_pc32_with_learned_correction():
    """The corrected S_hat preconditioner (per-node log-scales of the modal diagonal) in the
    FP32 chain's layout: with a random correction the state still matches the dense oracle
    at the FP64 bar, and its iteration count equals the FP64 run's with the same correction
    to within 0.5."""
    from paper_2105_01722_amd import gdw
    _say("case: pcg pc32 learned correction")
    n, N, p = 3, 12, 5
    Xm, Ym, c2, U0, V0 = _problem(n, N, p, True, True)
    dt, steps = 0.1 / (n * N), 2
    rng = np.random.default_rng(11)
    corr = (0.2 * rng.standard_normal((n * n, (N + 1) ** 2 - 1))).astype(np.float32)
    out = {}
    for prec in ("pc32", "fp64"):
        s = gdw.Solver(n, n, N, p, flux="upwind", xi=1.0, solver="pcg", coeff_variable=True,
                       mapped=True, pcg_rtol=1e-13, pcg_maxit=200, precision=prec)
        s.set_coeff(c2, Xm, Ym)
        s.set_precond_log(corr)
        s.set_state(U0, V0)
        s.run(dt, steps)
        U, V = s.get_state()
        out[prec] = (U.cpu().numpy(), V.cpu().numpy(), s.stats(check=False))
        s.close()
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="upwind"), Xm, Ym, c2)
    Uo, Vo = general.run(U0, V0, ops, dt, steps)
    Ug, Vg, st = out["pc32"]
    assert st["status"] == 0
    assert_close(Ug, Uo, 1e-12)
    assert_close(Vg, Vo, 1e-12)
    assert abs(st["mean_it_S"] - out["fp64"][2]["mean_it_S"]) <= 0.5


def test_pcg_pc32_unsupported():
    """GDW_MIXED_PC32 is refused where no FP32 chain exists: the constant-coefficient path,
    and N + 1 = 17 or N + 1 = 9 with p = 3 (per-node solve kernels), also inside a batch."""
    from paper_2105_01722_amd import gdw
    for kw in (dict(nx=2, ny=2, N=8, p=3, solver="fdm"),
               dict(nx=2, ny=2, N=16, p=5, solver="pcg", coeff_variable=True),
               dict(nx=2, ny=2, N=8, p=3, solver="pcg", coeff_variable=True)):
        with pytest.raises(gdw.GdwError) as ei:
            gdw.Solver(flux="upwind", precision="pc32", **kw)
        assert ei.value.status == gdw.GDW_EUNSUPPORTED
    with pytest.raises(gdw.GdwError) as ei:
        gdw.Batch([dict(nx=2, ny=2, N=16, p=5, flux="upwind", solver="pcg",
                        coeff_variable=True, precision="pc32")])
    assert ei.value.status == gdw.GDW_EUNSUPPORTED


def test_pcg_mixed_unsupported_size():
    """Mixed precision needs N + 1 in {9, 13, 17}: other sizes are refused at creation."""
    from paper_2105_01722_amd import gdw
    with pytest.raises(gdw.GdwError) as ei:
        gdw.Solver(2, 2, 10, 5, flux="upwind", solver="pcg", coeff_variable=True,
                   precision="mixed")
    assert ei.value.status == gdw.GDW_EUNSUPPORTED
