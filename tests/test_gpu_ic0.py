"""GPU parity of the IC(0) baseline (Sec. 7.1's incomplete Cholesky preconditioner)
against the oracle, through the C ABI (gdw_ic0_solve).

Bars: per element the IC(0)-PCG iteration count equals the oracle's within one (the stop
test compares two rounding-close residual norms), and the solution matches the dense
direct solve within 10 rtol cond(A) (the recurrence residual bound of CG at rtol).
"""
import sys

import numpy as np
import pytest

from oracle import general, ic0
from paper_2105_01722_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _setup(n, N, p, mapped):
    import torch
    from paper_2105_01722_amd import gdw
    X, Y = inputs.node_coords(n, n, N)
    c2 = inputs.c2_field(3, X, Y)
    Xm, Ym = inputs.mapped_coords(X, Y) if mapped else (X, Y)
    s = gdw.Solver(n, n, N, p, flux="upwind", xi=1.0, solver="pcg", coeff_variable=True,
                   mapped=mapped)
    s.set_coeff(c2, Xm, Ym)
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p), Xm, Ym, c2)
    nn = (N + 1) ** 2
    b = np.random.default_rng(11).standard_normal((n * n, nn))
    return s, ops, b, torch.tensor(b, device="cuda")


@pytest.mark.parametrize("n,N,p,mapped,op", [(2, 8, 3, True, 0), (2, 8, 3, True, 1),
                                             (3, 12, 5, True, 0), (2, 12, 5, True, 1),
                                             (2, 12, 5, False, 1), (2, 16, 7, True, 0)])
def test_ic0_matches_oracle(n, N, p, mapped, op):
    _say("case: ic0", n, N, p, mapped, op)
    s, ops, b, bg = _setup(n, N, p, mapped)
    rtol = 1e-12
    x, its = s.ic0_solve(op, bg, rtol=rtol, maxit=300)
    x, its = x.cpu().numpy(), its.cpu().numpy()
    s.close()
    P = ic0.stencil(N, p)
    for e in range(n * n):
        A = ic0.element_systems(ops, op)[e]
        _, ito, _ = ic0.ic0_pcg(A, b[e], P, rtol, 300)
        assert abs(int(its[e]) - ito) <= 1, (e, its[e], ito)
        xd = np.linalg.solve(A, b[e])
        err = np.linalg.norm(x[e] - xd) / np.linalg.norm(xd)
        assert err <= 10 * rtol * np.linalg.cond(A), (e, err)


def test_ic0_maxit_and_zero_rhs():
    """maxit reached is ENOCONV naming an element (every kernel still finishes); a zero
    right-hand side gives x = 0 in 0 iterations."""
    _say("case: ic0 maxit / zero rhs")
    import torch
    from paper_2105_01722_amd import gdw
    s, ops, b, bg = _setup(2, 8, 3, True)
    with pytest.raises(gdw.GdwError) as ex:
        s.ic0_solve(0, bg, rtol=1e-14, maxit=1)
    assert ex.value.status == gdw.GDW_ENOCONV
    x, its = s.ic0_solve(1, torch.zeros_like(bg))
    assert (its.cpu() == 0).all() and (x.cpu() == 0).all()
    s.close()
