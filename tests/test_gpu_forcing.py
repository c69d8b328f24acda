"""GPU parity of the source term (gdw_set_forcing) against the FP64 oracle, through the
C ABI, on the constant-coefficient path and on the PCG path (mapped elements, variable c^2).

Bars: FP64 nodal state relative l2 <= 1e-12 against the oracle (the periodic tests' bar),
FP32 storage <= 1e-6; a manufactured solution converges on the GPU path as in the oracle;
the source's clock continues across gdw_run calls and restarts at gdw_set_state; in a
batch (one captured step replayed) every member equals its solo run (constant-coefficient
members bitwise, PCG members within 1e-12).
"""
import sys

import numpy as np
import pytest

from oracle import dg2d, general
from paper_2105_01722_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


from _cmp import assert_close, rel as _rel, relmax as _relmax  # noqa: E402


def _solver(prob, precision="fp64"):
    from paper_2105_01722_amd import gdw
    s = gdw.Solver(prob.nx, prob.ny, prob.N, prob.p, c2=prob.c2, flux=prob.flux, xi=prob.xi,
                   precision=precision, Lx=prob.Lx, Ly=prob.Ly, x0=prob.x0, y0=prob.y0,
                   bc=prob.bc)
    return s


def _terms(prob, nterms, seed):
    X, Y = dg2d.node_coords(prob)
    out = []
    for k in range(nterms):
        g = inputs.fourier_field(inputs.fourier_modes(seed + k, kmax=3), X, Y)
        out.append((g, 3.0 + 2.0 * k, 0.3 * k))
    return out


@pytest.mark.parametrize("nx,ny,N,p,flux,nterms,bc", [
    (5, 3, 8, 3, "upwind", 1, ("periodic",) * 4),
    (3, 3, 16, 5, "upwind", 3, ("periodic",) * 4),
    (7, 2, 12, 5, "central", 2, ("dirichlet",) * 4),
    (2, 2, 10, 7, "upwind", 4, ("neumann", "neumann", "dirichlet", "dirichlet")),
])
def test_forcing_matches_oracle_fp64(nx, ny, N, p, flux, nterms, bc):
    _say("case: forcing fp64", nx, ny, N, p, flux, nterms, bc)
    base = dg2d.CartProblem(nx=nx, ny=ny, N=N, p=p, flux=flux, c2=1.2, xi=np.sqrt(1.2),
                            Lx=1.1, Ly=0.9, bc=bc)
    terms = _terms(base, nterms, 40)
    prob = dg2d.CartProblem(**{**base.__dict__, "forcing": tuple(terms)})
    X, Y = dg2d.node_coords(prob)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=3), X, Y)
    V0 = np.zeros_like(U0)
    dt = 0.1 * min(prob.hx, prob.hy)
    s = _solver(prob)
    try:
        s.set_state(U0, V0)
        s.set_forcing(terms)
        s.run(dt, 4)
        s.run(dt, 3)                                    # the clock continues
        Ug, Vg = (x.cpu().numpy() for x in s.get_state())
    finally:
        s.close()
    Uo, Vo = dg2d.run(U0, V0, dg2d.CartOps(prob), dt, 7)
    assert_close(Ug, Uo, 1e-12)
    assert_close(Vg, Vo, 1e-12)


def test_forcing_fp32_within_1e6():
    _say("case: forcing fp32")
    base = dg2d.CartProblem(nx=9, ny=3, N=12, p=5, flux="upwind")
    terms = _terms(base, 2, 50)
    prob = dg2d.CartProblem(**{**base.__dict__, "forcing": tuple(terms)})
    X, Y = dg2d.node_coords(prob)
    U0 = inputs.fourier_field(inputs.fourier_modes(4, kmax=3), X, Y)
    dt = 0.1 * prob.hx
    s = _solver(prob, "fp32")
    try:
        s.set_state(U0, np.zeros_like(U0))
        s.set_forcing(terms)
        s.run(dt, 6)
        Ug = s.get_state()[0].cpu().numpy()
    finally:
        s.close()
    Uo, _ = dg2d.run(U0, np.zeros_like(U0), dg2d.CartOps(prob), dt, 6)
    assert_close(Ug, Uo, 1e-6)


def test_manufactured_solution_converges_on_gpu():
    """u = sin(omega t) sin(2 pi x) sin(2 pi y), c^2 = 1.3, on the periodic unit square:
    f = (8 pi^2 c^2 - omega^2) sin(omega t) g.  p = 5, N = 10: the L2 error at t = 0.5
    falls at about the design order (> 5) when n doubles from 4 to 8."""
    _say("case: manufactured solution")
    omega, c2, T = 5.0, 1.3, 0.5
    errs = []
    for n in (4, 8):
        prob0 = dg2d.CartProblem(nx=n, ny=n, N=10, p=5, flux="upwind", c2=c2, xi=np.sqrt(c2))
        X, Y = dg2d.node_coords(prob0)
        g = np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
        amp = 8 * np.pi ** 2 * c2 - omega ** 2
        steps = int(np.ceil(T / (0.05 * prob0.hx)))
        s = _solver(prob0)
        try:
            s.set_state(np.zeros_like(g), omega * g)
            s.set_forcing([(amp * g, omega, 0.0)])
            s.run(T / steps, steps)
            U = s.get_state()[0].cpu().numpy()
        finally:
            s.close()
        errs.append(dg2d.l2_error(U, prob0, lambda x, y: np.sin(omega * T)
                                  * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)))
    rate = np.log2(errs[0] / errs[1])
    _say("  errors", errs, "rate", rate)
    assert errs[1] < 1e-7 and rate > 5.0


def test_clock_restarts_at_set_state_and_zero_terms_remove_the_source():
    from paper_2105_01722_amd import gdw
    _say("case: forcing clock")
    prob = dg2d.CartProblem(nx=4, ny=3, N=8, p=3, flux="upwind")
    terms = _terms(prob, 2, 60)
    X, Y = dg2d.node_coords(prob)
    U0 = inputs.fourier_field(inputs.fourier_modes(5, kmax=3), X, Y)
    V0 = np.zeros_like(U0)
    dt = 0.1 * prob.hx
    s = _solver(prob)
    try:
        s.set_forcing(terms)
        s.set_state(U0, V0)
        s.run(dt, 5)
        A = s.get_state()[0].cpu().numpy()
        s.set_state(U0, V0)                              # the clock restarts at 0
        s.run(dt, 3)
        s.run(dt, 2)
        B = s.get_state()[0].cpu().numpy()
        np.testing.assert_array_equal(A, B)
        s.set_forcing([])
        s.set_state(U0, V0)
        s.run(dt, 5)
        C = s.get_state()[0].cpu().numpy()
    finally:
        s.close()
    s2 = _solver(prob)
    try:
        s2.set_state(U0, V0)
        s2.run(dt, 5)
        D = s2.get_state()[0].cpu().numpy()
    finally:
        s2.close()
    np.testing.assert_array_equal(C, D)
    assert _rel(A, D) > 1e-6


def test_forcing_errors():
    from paper_2105_01722_amd import gdw
    _say("case: forcing errors")
    prob = dg2d.CartProblem(nx=2, ny=2, N=8, p=3, flux="upwind")
    s = _solver(prob)
    try:
        g = np.zeros((2, 2, 9, 9))
        with pytest.raises(gdw.GdwError) as ei:
            s.set_forcing([(g, 1.0, 0.0)] * 5)
        assert ei.value.status == gdw.GDW_EINVAL
        with pytest.raises(gdw.GdwError) as ei:
            s.set_forcing([(g, float("nan"), 0.0)])
        assert ei.value.status == gdw.GDW_EINVAL
    finally:
        s.close()


# ---- PCG path -------------------------------------------------------------------------
def _pcg(n, N, p, Xm, Ym, c2, bc=("periodic",) * 4, rtol=1e-13, precision="fp64"):
    from paper_2105_01722_amd import gdw
    s = gdw.Solver(n, n, N, p, flux="upwind", xi=1.0, solver="pcg", coeff_variable=True,
                   mapped=True, pcg_rtol=rtol, bc=bc, precision=precision)
    s.set_coeff(c2, Xm, Ym)
    return s


@pytest.mark.parametrize("n,N,p,nterms,bc", [(3, 12, 5, 2, ("periodic",) * 4),
                                             (3, 8, 3, 1, ("dirichlet",) * 4),
                                             (2, 16, 5, 3, ("neumann", "neumann", "periodic", "periodic")),
                                             (3, 7, 5, 1, ("periodic",) * 4)])
def test_pcg_forcing_matches_dense_oracle(n, N, p, nterms, bc):
    """Register-operator kernels (N + 1 = 13, 9, 17) and the row layout (N = 7)."""
    _say("case: pcg forcing", n, N, p, nterms, bc)
    X, Y = inputs.node_coords(n, n, N)
    Xm, Ym = inputs.mapped_coords(X, Y)
    c2 = inputs.c2_field(3, X, Y)
    terms = [(inputs.fourier_field(inputs.fourier_modes(70 + k, kmax=3), Xm, Ym), 4.0 + k, 0.5 * k)
             for k in range(nterms)]
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=3), Xm, Ym)
    V0 = np.zeros_like(U0)
    dt = 0.1 / (n * N)
    s = _pcg(n, N, p, Xm, Ym, c2, bc)
    try:
        s.set_forcing(terms)
        s.set_state(U0, V0)
        s.run(dt, 2)
        s.run(dt, 1)                                    # the device clock continues
        Ug, Vg = (x.cpu().numpy() for x in s.get_state())
        assert s.stats(check=False)["status"] == 0
    finally:
        s.close()
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="upwind", bc=bc,
                                            forcing=tuple(terms)), Xm, Ym, c2)
    Uo, Vo = general.run(U0, V0, ops, dt, 3)
    assert_close(Ug, Uo, 1e-12)
    assert_close(Vg, Vo, 1e-12)


def test_pcg_manufactured_solution_on_curved_mesh_converges():
    """u = sin(omega t) sin(2 pi x) sin(2 pi y) with c^2 = 1 + 0.25 sin(2 pi x) cos(2 pi y)
    on the curved mesh, the exact solution of the forced PDE: p = 5, N = 12, the nodal
    error at t = 0.2 falls at > 5 when n doubles from 4 to 8 (PCG at rtol 1e-12)."""
    _say("case: pcg manufactured")
    omega, T = 5.0, 0.2
    tp = 2 * np.pi
    errs = []
    for n in (4, 8):
        N, p = 12, 5
        X, Y = inputs.node_coords(n, n, N)
        Xm, Ym = inputs.mapped_coords(X, Y)
        phi = np.sin(tp * Xm) * np.sin(tp * Ym)
        c2 = 1.0 + 0.25 * np.sin(tp * Xm) * np.cos(tp * Ym)
        grad = (0.25 * tp * np.cos(tp * Xm) * np.cos(tp * Ym) * tp * np.cos(tp * Xm) * np.sin(tp * Ym)
                - 0.25 * tp * np.sin(tp * Xm) * np.sin(tp * Ym) * tp * np.sin(tp * Xm) * np.cos(tp * Ym))
        g = -omega ** 2 * phi + 2 * tp ** 2 * c2 * phi - grad
        steps = int(np.ceil(T / (0.1 / (n * N))))        # dt <= 0.1 h (RK4 stable at p = 5)
        s = _pcg(n, N, p, Xm, Ym, c2, rtol=1e-12)
        try:
            s.set_state(np.zeros_like(phi), omega * phi)
            s.set_forcing([(g, omega, 0.0)])
            s.run(T / steps, steps)
            U = s.get_state()[0].cpu().numpy()
        finally:
            s.close()
        errs.append(np.abs(U - np.sin(omega * T) * phi).max())
    rate = np.log2(errs[0] / errs[1])
    _say("  errors", errs, "rate", rate)
    assert errs[1] < 1e-5 and rate > 5.0


def test_batch_with_source_terms_equals_solo_runs():
    """Forced and unforced members in the same classes; two runs (3 + 2 steps) so the
    captured step's weights kernel must advance each member's clock."""
    from paper_2105_01722_amd import gdw
    _say("case: batch with source terms")
    probs = [dict(nx=3, ny=2, N=8, p=3, flux="upwind", precision="fp64"),
             dict(nx=2, ny=2, N=8, p=3, flux="upwind", precision="fp64"),
             dict(nx=4, ny=3, N=12, p=5, flux="upwind", precision="fp32",
                  bc=("dirichlet",) * 4),
             dict(nx=2, ny=2, N=12, p=5, flux="upwind", solver="pcg", coeff_variable=True,
                  mapped=True, pcg_rtol=1e-13),
             dict(nx=2, ny=3, N=12, p=5, flux="upwind", solver="pcg", coeff_variable=True,
                  mapped=True, pcg_rtol=1e-13)]
    forced = [True, False, True, True, False]

    def setup(s, i, kw):
        X, Y = inputs.node_coords(kw["nx"], kw["ny"], kw["N"])
        if kw.get("solver") == "pcg":
            Xm, Ym = inputs.mapped_coords(X, Y)
            s.set_coeff(inputs.c2_field(80 + i, X, Y), Xm, Ym)
            X, Y = Xm, Ym
        U0 = inputs.fourier_field(inputs.fourier_modes(90 + i, kmax=3), X, Y)
        s.set_state(U0, np.zeros_like(U0))
        if forced[i]:
            g = inputs.fourier_field(inputs.fourier_modes(95 + i, kmax=3), X, Y)
            s.set_forcing([(g, 4.0 + i, 0.1 * i), (0.5 * g, 9.0, -0.3)])

    dts = [0.1 / (max(kw["nx"], kw["ny"]) * kw["N"]) for kw in probs]
    b = gdw.Batch(probs)
    try:
        for i, kw in enumerate(probs):
            setup(b.problems[i], i, kw)
        b.run(dts, 3)
        b.run(dts, 2)
        got = [tuple(x.cpu().numpy() for x in b.problems[i].get_state()) for i in range(len(probs))]
    finally:
        b.close()
    for i, kw in enumerate(probs):
        s = gdw.Solver(**kw)
        try:
            setup(s, i, kw)
            s.run(dts[i], 3)
            s.run(dts[i], 2)
            U, V = (x.cpu().numpy() for x in s.get_state())
        finally:
            s.close()
        Ub, Vb = got[i]
        if kw.get("solver") == "pcg":
            assert_close(Ub, U, 1e-12)
            assert_close(Vb, V, 1e-12)
        else:
            np.testing.assert_array_equal(Ub, U)
            np.testing.assert_array_equal(Vb, V)


def test_pcg_mixed_precision_with_source():
    """Mixed-precision PCG (FP32 inner iterations, FP64 refinement) with a source term
    and walls, against the dense oracle at the mixed path's bar (1e-10)."""
    _say("case: pcg mixed with source")
    n, N, p = 3, 12, 5
    bc = ("dirichlet", "dirichlet", "neumann", "neumann")
    X, Y = inputs.node_coords(n, n, N)
    Xm, Ym = inputs.mapped_coords(X, Y)
    c2 = inputs.c2_field(3, X, Y)
    terms = [(inputs.fourier_field(inputs.fourier_modes(75, kmax=3), Xm, Ym), 6.0, 0.2)]
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=3), Xm, Ym)
    dt = 0.1 / (n * N)
    s = _pcg(n, N, p, Xm, Ym, c2, bc, precision="mixed")
    try:
        s.set_forcing(terms)
        s.set_state(U0, np.zeros_like(U0))
        s.run(dt, 3)
        Ug, Vg = (x.cpu().numpy() for x in s.get_state())
        st = s.stats(check=False)
        assert st["status"] == 0 and st["mean_refine"] >= 1.0
    finally:
        s.close()
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p, flux="upwind", bc=bc,
                                            forcing=tuple(terms)), Xm, Ym, c2)
    Uo, Vo = general.run(U0, np.zeros_like(U0), ops, dt, 3)
    assert_close(Ug, Uo, 1e-10)
    assert_close(Vg, Vo, 1e-10)