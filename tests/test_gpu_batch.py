"""Batched time loop (gdw_batch_*) against the same problems run one by one.

Each problem of a batch advances exactly as gdw_run advances it alone: the grouped
stage kernels run the same per-element arithmetic.  Bars: constant-coefficient problems
bitwise equal to their solo runs (the per-element arithmetic does not depend on the
tile size); PCG problems within 1e-12 relative l2 of their solo runs (the block size
chosen by the tuner may split the matrix rows differently, which changes the rounding of
the row sums) and of the FP64 oracle for one of them.
"""
import sys

import numpy as np
import pytest

from oracle import general
from paper_2105_01722_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


from _cmp import assert_close, rel as _rel  # noqa: E402


PROBLEMS = [
    dict(nx=3, ny=2, N=8, p=3, flux="upwind", precision="fp64"),
    dict(nx=2, ny=3, N=12, p=5, flux="upwind", precision="fp64"),
    dict(nx=3, ny=3, N=16, p=5, flux="central", precision="fp64"),
    dict(nx=2, ny=2, N=16, p=7, flux="upwind", precision="fp32"),
    dict(nx=4, ny=3, N=8, p=5, flux="upwind", precision="fp32"),
    dict(nx=2, ny=2, N=10, p=5, flux="upwind", precision="fp64"),        # generic N+1
    dict(nx=3, ny=3, N=8, p=3, flux="upwind", solver="pcg", coeff_variable=True, mapped=True,
         pcg_rtol=1e-13),
    dict(nx=2, ny=3, N=12, p=5, flux="upwind", solver="pcg", coeff_variable=True, mapped=True,
         pcg_rtol=1e-13),
    dict(nx=3, ny=2, N=12, p=5, flux="upwind", solver="pcg", coeff_variable=True, pcg_rtol=1e-13),
    dict(nx=2, ny=2, N=16, p=5, flux="upwind", solver="pcg", coeff_variable=True, mapped=True,
         pcg_rtol=1e-13),
    dict(nx=2, ny=3, N=12, p=7, flux="upwind", solver="pcg", coeff_variable=True, mapped=True,
         pcg_rtol=1e-13),
    # the streamed family (N+1 = 17, p = 7): a mapped and a Cartesian member, so that the
    # class's M_J solves cover only one of them
    dict(nx=2, ny=2, N=16, p=7, flux="upwind", solver="pcg", coeff_variable=True, mapped=True,
         pcg_rtol=1e-13),
    dict(nx=3, ny=2, N=16, p=7, flux="upwind", solver="pcg", coeff_variable=True, pcg_rtol=1e-13),
    # members with walls, grouped with periodic members of the same class
    dict(nx=3, ny=2, N=8, p=3, flux="upwind", precision="fp64", bc=("dirichlet",) * 4),
    dict(nx=4, ny=3, N=8, p=5, flux="upwind", precision="fp32",
         bc=("neumann", "neumann", "dirichlet", "dirichlet")),
    dict(nx=2, ny=3, N=12, p=5, flux="upwind", solver="pcg", coeff_variable=True, mapped=True,
         pcg_rtol=1e-13, bc=("dirichlet", "dirichlet", "periodic", "periodic")),
]


def _inputs(i, kw):
    nx, ny, N = kw["nx"], kw["ny"], kw["N"]
    X, Y = inputs.node_coords(nx, ny, N)
    c2 = Xm = Ym = None
    if kw.get("coeff_variable"):
        c2 = inputs.c2_field(100 + i, X, Y)
    if kw.get("mapped"):
        Xm, Ym = inputs.mapped_coords(X, Y)
    Xu, Yu = (Xm, Ym) if Xm is not None else (X, Y)
    U0 = inputs.fourier_field(inputs.fourier_modes(200 + i, kmax=3), Xu, Yu)
    V0 = 0.3 * inputs.fourier_field(inputs.fourier_modes(300 + i, kmax=3), Xu, Yu)
    return c2, Xm, Ym, U0, V0


def _prepare(s, i, kw):
    c2, Xm, Ym, U0, V0 = _inputs(i, kw)
    if kw.get("solver") == "pcg":
        s.set_coeff(c2, Xm, Ym)
    s.set_state(U0, V0)


def _dt(kw, cfl=0.05):
    return cfl / (max(kw["nx"], kw["ny"]) * kw["N"])


def _solo(i, kw, dt, steps):
    from paper_2105_01722_amd import gdw
    s = gdw.Solver(**kw)
    _prepare(s, i, kw)
    s.run(dt, steps)
    U, V = s.get_state()
    st = s.stats()
    s.close()
    return U.cpu().numpy(), V.cpu().numpy(), st


def test_batch_equals_solo_runs_and_rebuilds_on_new_dt():
    from paper_2105_01722_amd import gdw
    _say("case: batch of %d mixed problems" % len(PROBLEMS))
    b = gdw.Batch(PROBLEMS)
    for i, kw in enumerate(PROBLEMS):
        _prepare(b.problems[i], i, kw)
    dts = [_dt(kw) for kw in PROBLEMS]
    b.tune(dts)
    plan = b.plan()
    _say(plan.split("candidates:")[0])
    assert "fdm n1=9" in plan and "pcg blocks n1=13" in plan
    assert "n1=17 (registers, p=5)" in plan and "n1=13 (registers, p=7)" in plan
    b.run(dts, 3)
    times = b.step_times()
    assert len(times) == 3 and all(t > 0 for t in times)
    dts2 = [0.7 * d for d in dts]
    b.run(dts2, 2)                    # a new dt: the graph is rebuilt
    assert len(b.step_times()) == 2
    got = []
    for i in range(len(PROBLEMS)):
        U, V = b.problems[i].get_state()
        st = b.problems[i].stats()
        assert st["steps_taken"] == 5
        got.append((U.cpu().numpy(), V.cpu().numpy()))
    b.close()
    for i, kw in enumerate(PROBLEMS):
        from paper_2105_01722_amd import gdw as g2
        s = g2.Solver(**kw)
        _prepare(s, i, kw)
        s.run(dts[i], 3)
        s.run(dts2[i], 2)
        U, V = s.get_state()
        s.close()
        U, V = U.cpu().numpy(), V.cpu().numpy()
        Ub, Vb = got[i]
        if kw.get("solver") == "pcg":
            eu, ev = _rel(Ub, U), _rel(Vb, V)
            _say("  problem %d (pcg): rel U %.2e V %.2e" % (i, eu, ev))
            assert_close(Ub, U, 1e-12)
            assert_close(Vb, V, 1e-12)
        else:
            _say("  problem %d (fdm %s): max |diff| U %.2e V %.2e"
                 % (i, kw["precision"], np.abs(Ub - U).max(), np.abs(Vb - V).max()))
            np.testing.assert_array_equal(Ub, U)
            np.testing.assert_array_equal(Vb, V)


def test_batch_pcg_member_matches_oracle():
    from paper_2105_01722_amd import gdw
    kw = PROBLEMS[7]
    probs = [PROBLEMS[0], kw]
    b = gdw.Batch(probs)
    for i, k in enumerate(probs):
        _prepare(b.problems[i], 7 if i == 1 else 0, k)
    dts = [_dt(k) for k in probs]
    b.run(dts, 2)
    U, V = b.problems[1].get_state()
    b.close()
    c2, Xm, Ym, U0, V0 = _inputs(7, kw)
    prob = general.GenProblem(nx=kw["nx"], ny=kw["ny"], N=kw["N"], p=kw["p"], flux="upwind")
    ops = general.GenOps(prob, Xm, Ym, c2)
    Uo, Vo = general.run(U0, V0, ops, dts[1], 2)
    eu, ev = _rel(U.cpu().numpy(), Uo), _rel(V.cpu().numpy(), Vo)
    _say("  batch pcg member vs oracle: U %.2e V %.2e" % (eu, ev))
    assert_close(U.cpu().numpy(), Uo, 1e-12)
    assert_close(V.cpu().numpy(), Vo, 1e-12)


def test_batch_reuses_tuned_shapes():
    """The tuner's launch shapes are kept for the life of the process, keyed by architecture,
    path, arithmetic, kernel family and member sizes: a second batch with the same classes
    takes them untimed (its plan marks every tuned class cached) and advances its problems
    bitwise as the first batch did."""
    from paper_2105_01722_amd import gdw
    probs = [PROBLEMS[0], PROBLEMS[3],
             dict(nx=2, ny=2, N=12, p=5, flux="upwind", solver="pcg", coeff_variable=True,
                  mapped=True, precision="mixed", pcg_rtol=1e-12)]
    plans, states = [], []
    for rep in range(2):
        _say("case: tuned shapes, batch %d" % rep)
        b = gdw.Batch(probs)
        for i, kw in enumerate(probs):
            _prepare(b.problems[i], 40 + i, kw)
        dts = [_dt(kw) for kw in probs]
        b.tune(dts)
        plans.append(b.plan())
        b.run(dts, 2)
        states.append([tuple(x.cpu().numpy() for x in b.problems[i].get_state())
                       for i in range(len(probs))])
        b.close()
    cand = plans[1].split("candidates:")[1]
    _say(cand)
    assert cand.count("(cached)") == 3 and " ms" not in cand
    for (U0, V0), (U1, V1) in zip(states[0], states[1]):
        np.testing.assert_array_equal(U0, U1)
        np.testing.assert_array_equal(V0, V1)


def test_batch_pc32_members_equal_solo_runs():
    """Problems with the FP32 preconditioner chain (GDW_MIXED_PC32) form classes of their
    own beside FP64 members of the same family; each advances as its solo run (1e-12, as the
    other PCG members)."""
    from paper_2105_01722_amd import gdw
    base = dict(flux="upwind", solver="pcg", coeff_variable=True, pcg_rtol=1e-13)
    probs = [dict(nx=2, ny=3, N=12, p=5, mapped=True, precision="pc32", **base),
             dict(nx=3, ny=2, N=12, p=5, mapped=True, precision="fp64", **base),
             dict(nx=3, ny=3, N=8, p=5, precision="pc32", **base),
             dict(nx=2, ny=2, N=12, p=5, mapped=True, precision="pc32", **base)]
    b = gdw.Batch(probs)
    for i, kw in enumerate(probs):
        _prepare(b.problems[i], 60 + i, kw)
    dts = [_dt(kw) for kw in probs]
    b.run(dts, 3)
    plan = b.plan()
    _say(plan.split("candidates:")[0])
    assert plan.count("FP32 chain") == 2
    got = [tuple(x.cpu().numpy() for x in b.problems[i].get_state()) for i in range(len(probs))]
    b.close()
    for i, kw in enumerate(probs):
        s = gdw.Solver(**kw)
        _prepare(s, 60 + i, kw)
        s.run(dts[i], 3)
        U, V = (x.cpu().numpy() for x in s.get_state())
        s.close()
        assert_close(got[i][0], U, 1e-12)
        assert_close(got[i][1], V, 1e-12)
