"""Pins of the oracle's semi-discrete operator against the claims of the paper's
dispersion analysis (Sec. 4) and spectral-radius study (Sec. 5).

The paper reports both only in figures, so the pins are the properties it states:
  * Sec. 5: the spectral radius grows linearly with p for the central, the alternating
    and the upwind flux, with periodic ends and with a Dirichlet left / Neumann right end (standard DG
    grows like p^2); rho is proportional to 1/h, so rho h depends on p and not on N;
  * Sec. 4: the central and the alternating flux give purely imaginary eigenvalues (no
    numerical damping), the upwind flux none with positive real part; the physical mode of a well-resolved
    Bloch wave has a phase error that is small and falls as p grows.

The 1D operator is the oracle's 2D scheme restricted to y-independent states (the
invariant subspace used by test_oracle_convergence.py), assembled column by column.
"""
import numpy as np
import pytest

from oracle import dg2d
from test_oracle_convergence import _strip_operator

PERIODIC = ("periodic",) * 4
DIR_NEU = ("neumann", "dirichlet", "periodic", "periodic")   # Neumann right, Dirichlet left


def _spectrum(n, N, p, flux, bc=PERIODIC):
    prob = dg2d.CartProblem(nx=n, ny=1, N=N, p=p, flux=flux, bc=bc)
    L, worst = _strip_operator(prob, dg2d.CartOps(prob))
    assert worst < 1e-10
    return np.linalg.eigvals(L), prob


@pytest.mark.parametrize("flux", ["central", "upwind", "alternating"])
@pytest.mark.parametrize("bc", [PERIODIC, DIR_NEU])
def test_spectral_radius_linear_in_p(flux, bc):
    rh = {}
    for N in (9, 19):
        for p in (3, 5, 7, 9):
            ev, prob = _spectrum(3, N, p, flux, bc)
            rh[N, p] = np.abs(ev).max() * prob.hx
    for N in (9, 19):
        seq = [rh[N, p] for p in (3, 5, 7, 9)]
        assert all(b > a for a, b in zip(seq, seq[1:])), seq       # grows with p
        # linear growth through the origin gives rho(9) / rho(3) = 3, p^2 growth gives 9
        assert seq[-1] / seq[0] <= 3.0, seq
    for p in (3, 5, 7, 9):                                       # rho ~ 1/h
        assert abs(rh[9, p] - rh[19, p]) <= 0.1 * rh[19, p]


@pytest.mark.parametrize("p", [1, 3, 5, 7])
def test_central_flux_spectrum_is_imaginary_upwind_has_no_growth(p):
    """Away from zero: central Re = 0 to rounding, upwind Re < 0.  The zero eigenvalue is
    multiple and defective (for instance the steady constant u and the mode u = b t,
    v = b form a Jordan block), and eigvals splits a Jordan block of size two by about
    sqrt(eps) rho; those eigenvalues are checked to be that small and set apart.  A
    flipped sign of the upwind tau term gives Re / rho of order one.  (Any alpha with
    beta = tau = 0 conserves the energy, so this test does not see alpha.)"""
    for flux in ("central", "alternating", "upwind"):
        ev, _ = _spectrum(4, 9, p, flux)
        rho = np.abs(ev).max()
        zero = np.abs(ev) <= 1e-6 * rho
        assert zero.sum() >= 2
        rest = ev[~zero]
        if flux != "upwind":
            assert np.abs(rest.real).max() <= 1e-12 * rho
        else:
            assert rest.real.max() <= 1e-12 * rho


@pytest.mark.parametrize("flux", ["central", "upwind", "alternating"])
def test_physical_mode_phase_error_falls_with_p(flux):
    """Bloch waves exp(i kappa x) on the periodic unit interval (4 elements, N = 9, 36
    cells): for kappa = 2 pi and 4 pi the eigenvalue nearest to i kappa has a relative
    phase error below 1e-5 for p >= 3 that falls as p grows, and (upwind) a damping
    |Re| / kappa below 1e-5."""
    errs = {}
    for p in (1, 3, 5):
        ev, _ = _spectrum(4, 9, p, flux)
        for m in (1, 2):
            k = 2 * np.pi * m
            lam = ev[np.argmin(np.abs(ev - 1j * k))]
            errs[p, m] = abs(lam.imag - k) / k
            if p >= 3:
                assert errs[p, m] < 1e-5
                assert abs(lam.real) / k < 1e-5
    for m in (1, 2):
        assert errs[1, m] > errs[3, m] > errs[5, m]
