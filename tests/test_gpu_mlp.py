"""GPU checks of the learned preconditioner correction against the FP64 reference.

Bars (FP16 forward products with FP32 accumulation): forward outputs within 2e-2
relative l2 of the FP64 reference; gradients within 5e-2 relative l2 (FP16 rounding of
activations and weights in the forward pass propagates into them); the first Adam
step moves every parameter with a clear gradient by -lr g / (|g| + eps); the solver-side
training data matches the oracle's definition; corrections never change the converged
solution (dense-oracle parity at tight tolerance) and a failing correction falls back
to the plain preconditioner.
"""
import sys

import numpy as np
import pytest

from oracle import general, mlp as omlp, pcg
from paper_2105_01722_amd import inputs

pytestmark = pytest.mark.gpu
NI, H, K = 64, 128, 168


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


from _cmp import assert_close, rel as _rel  # noqa: E402


def _net(seed=0):
    from paper_2105_01722_amd import gdw
    return gdw.Mlp(NI, H, K, seed=seed, max_batch=512)


def test_forward_matches_reference():
    _say("case: mlp forward")
    net = _net(1)
    th = net.get_params().astype(np.float64)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((300, NI))
    out = net.forward(x.astype(np.float32)).cpu().numpy()
    ref, _ = omlp.forward(th, x, NI, H, K)
    assert_close(out, ref, 2e-2, max_bar=5e-2)
    net.close()


def test_gradient_matches_reference():
    _say("case: mlp gradient")
    net = _net(2)
    th = net.get_params().astype(np.float64)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((200, NI))
    y = 0.1 * rng.standard_normal((200, K))
    g, loss = net.grad(x.astype(np.float32), y.astype(np.float32))
    lref, gref = omlp.loss_and_grad(th, x, y, NI, H, K)
    assert abs(loss - lref) <= 2e-2 * lref
    assert_close(g.cpu().numpy(), gref, 5e-2, max_bar=2e-1)
    net.close()


def test_first_adam_step_formula():
    _say("case: mlp adam")
    net = _net(3)
    th0 = net.get_params().astype(np.float64)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((128, NI)).astype(np.float32)
    y = (0.1 * rng.standard_normal((128, K))).astype(np.float32)
    _, gref = omlp.loss_and_grad(th0, x, y, NI, H, K)
    net.train(x, y, epochs=1, batch=128, lr=1e-3)
    d = net.get_params().astype(np.float64) - th0
    # first step with bias correction: -lr g / (|g| + eps), eps = 1e-8; compared where the
    # gradient is well above the FP16 forward-pass noise
    big = np.abs(gref) > 1e-3 * np.abs(gref).max()
    np.testing.assert_allclose(d[big], -1e-3 * gref[big] / (np.abs(gref[big]) + 1e-8),
                               rtol=2e-3, atol=2e-7)
    net.close()


def test_training_reduces_loss():
    _say("case: mlp training")
    net = _net(4)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2048, NI)).astype(np.float32)
    W = rng.standard_normal((NI, K)) / 8
    y = np.tanh(x @ W).astype(np.float32) * 0.1
    losses = net.train(x, y, epochs=30, batch=256, lr=1e-3)
    assert losses[-1] < 0.2 * losses[0]
    net.close()


def _gpu_problem(n, N, p, mapped, rtol=1e-13, maxit=200):
    from paper_2105_01722_amd import gdw
    X, Y = inputs.node_coords(n, n, N)
    c2 = inputs.c2_field(3, X, Y)
    Xm, Ym = inputs.mapped_coords(X, Y) if mapped else (X, Y)
    s = gdw.Solver(n, n, N, p, flux="upwind", xi=1.0, solver="pcg", coeff_variable=True,
                   mapped=mapped, pcg_rtol=rtol, pcg_maxit=maxit)
    s.set_coeff(c2, Xm, Ym)
    return s, Xm, Ym, c2


def test_precond_data_matches_oracle():
    _say("case: precond data")
    n, N, p = 3, 8, 5
    s, Xm, Ym, c2 = _gpu_problem(n, N, p, mapped=True)
    smp, tgt = s.precond_data()
    s.close()
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p), Xm, Ym, c2)
    np.testing.assert_allclose(smp.cpu().numpy(), omlp.coefficient_samples(c2, N, p), atol=1e-6)
    ref = omlp.modal_targets(ops)
    np.testing.assert_allclose(tgt.cpu().numpy(), ref, atol=2e-6 + 1e-5 * np.abs(ref).max())


def _run(s, U0, V0, dt, steps):
    s.set_state(U0, V0)
    s.run(dt, steps)
    U, V = s.get_state()
    st = s.stats(check=False)
    return U.cpu().numpy(), V.cpu().numpy(), st


def test_corrections_keep_the_solution_and_fallback():
    """Analytic control (exact modal diagonal), a NaN correction (sanitised to the plain
    one) and a wild correction with a small iteration limit (falls back to plain): the
    state matches the dense oracle in every case."""
    _say("case: corrections")
    n, N, p = 3, 8, 5
    s, Xm, Ym, c2 = _gpu_problem(n, N, p, mapped=True, maxit=80)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=3), Xm, Ym)
    V0 = np.zeros_like(U0)
    dt, steps = 0.1 / (n * N), 2
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p), Xm, Ym, c2)
    Uo, Vo = general.run(U0, V0, ops, dt, steps)
    Up, _, st_plain = _run(s, U0, V0, dt, steps)
    _, tgt = s.precond_data()
    with pytest.raises(ValueError):
        s.set_precond_log(tgt.reshape(-1)[:-1])   # one entry short: refused in the binding
    s.set_precond_log(tgt)
    Ua, _, st_exact = _run(s, U0, V0, dt, steps)
    bad = np.full(tgt.shape, np.nan, dtype=np.float32)
    s.set_precond_log(bad)
    Ub, _, st_nan = _run(s, U0, V0, dt, steps)
    s.set_precond_log(np.full(tgt.shape, 8.0, dtype=np.float32))
    Uw, _, st_wild = _run(s, U0, V0, dt, steps)
    s.close()
    for U, st in ((Up, st_plain), (Ua, st_exact), (Ub, st_nan), (Uw, st_wild)):
        assert st["status"] == 0
        assert_close(U, Uo, 1e-12)
    assert st_nan["mean_it_S"] == st_plain["mean_it_S"]
    assert st_exact["mean_it_S"] <= st_plain["mean_it_S"] + 0.5


def test_trained_network_end_to_end():
    """Train on the solver's own data of one coefficient field, apply to another: the
    PCG path still matches the dense oracle; iteration counts are reported."""
    _say("case: trained network")
    n, N, p = 4, 8, 5
    s, Xm, Ym, c2 = _gpu_problem(n, N, p, mapped=False)
    smp, tgt = s.precond_data()
    net = _net(5)
    net_k = (N + 1) ** 2 - 1
    if net_k != K:
        net.close()
        from paper_2105_01722_amd import gdw
        net = gdw.Mlp(NI, 32, net_k, seed=5, max_batch=512)
    losses = net.train(smp, tgt, epochs=50, batch=8, lr=1e-3)
    assert np.isfinite(losses).all()
    s.set_precond_mlp(net)
    U0 = inputs.fourier_field(inputs.fourier_modes(2, kmax=3), Xm, Ym)
    V0 = np.zeros_like(U0)
    dt = 0.1 / (n * N)
    Ug, _, st = _run(s, U0, V0, dt, 2)
    s.close()
    net.close()
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p), Xm, Ym, c2)
    Uo, _ = general.run(U0, V0, ops, dt, 2)
    assert st["status"] == 0
    assert_close(Ug, Uo, 1e-12)
