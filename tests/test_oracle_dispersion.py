"""The Bloch (dispersion) analysis of Sec. 4 as an oracle harness (oracle/analysis.py),
pinned to the operator it analyses and to the paper's statements.

  * brute force: the symbol's eigenvalues at theta = 2 pi m / n are, together, exactly the
    spectrum of the assembled periodic operator on n elements;
  * Sec. 4: the conservative fluxes (central, alternating) give purely imaginary
    dispersion relations (no damping of any mode); the upwind flux leaves the physical
    pair +-i K at small K undamped to 1e-6 K and damps every spurious mode;
  * the physical mode: its phase error at K H = 2 pi / 8 falls quickly with p (the
    paper's figures show it converging to the exact relation), and for p = 3 with N = 9
    (the paper's setting of its dispersion figures) it is below 1e-6.
"""
import numpy as np
import pytest

from oracle import analysis, dg2d
from test_oracle_convergence import _strip_operator


@pytest.mark.parametrize("flux", ["central", "upwind", "alternating"])
def test_symbol_reproduces_the_periodic_spectrum(flux):
    n, N, p = 4, 6, 3
    prob = dg2d.CartProblem(nx=n, ny=1, N=N, p=p, flux=flux, Lx=float(n), Ly=1.0)
    L, _ = _strip_operator(prob, dg2d.CartOps(prob))
    want = np.sort_complex(np.round(np.linalg.eigvals(L), 8))
    lam = analysis.bloch_eigenvalues(N, p, flux, 2 * np.pi * np.arange(n) / n, H=1.0)
    got = np.sort_complex(np.round(lam.ravel(), 8))
    scale = np.abs(want).max()
    # the zero eigenvalue is defective (a Jordan block): both sides split it by ~sqrt(eps)
    far = np.abs(want) > 1e-5 * scale
    assert far.sum() == (np.abs(got) > 1e-5 * scale).sum()
    assert np.abs(got[np.abs(got) > 1e-5 * scale] - want[far]).max() <= 1e-7 * scale


@pytest.mark.parametrize("flux", ["central", "alternating", "upwind"])
def test_dispersion_relation_damping(flux):
    N, p, H = 9, 3, 1.0
    thetas = np.linspace(-np.pi, np.pi, 41)
    lam = analysis.bloch_eigenvalues(N, p, flux, thetas, H)
    rho = np.abs(lam).max()
    if flux == "upwind":
        assert lam.real.max() <= 1e-10 * rho
        # at a small wavenumber the physical pair +-i K is (almost) undamped and every
        # spurious mode is damped
        t = np.argmin(np.abs(thetas - 2 * np.pi / 41 * 4))
        ev, K = lam[t], abs(thetas[t]) / H
        phys = [np.argmin(np.abs(ev - 1j * K)), np.argmin(np.abs(ev + 1j * K))]
        assert np.abs(ev[phys].real).max() <= 1e-6 * K
        others = np.delete(ev, phys)
        others = others[np.abs(others) > 1e-6 * rho]
        assert (-others.real / np.abs(others)).min() > 1e-5
    else:
        big = np.abs(lam) > 1e-6 * rho
        assert np.abs(lam.real[big]).max() <= 1e-9 * rho


@pytest.mark.parametrize("flux", ["central", "upwind", "alternating"])
def test_physical_mode_converges_with_p(flux):
    N, H = 9, 1.0
    K = 2 * np.pi / 8 / H
    err = {p: abs(analysis.physical_mode(N, p, flux, K, H) - 1j * K) / K for p in (1, 3, 5)}
    assert err[1] > err[3] > err[5]
    assert err[3] < 1e-6
