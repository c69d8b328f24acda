"""Pins of the FP64 reference network and its training data (no paper passage: this
part is a spec addition).  Backpropagation is checked against central finite
differences; Adam against a hand-evaluated first step; the coefficient samples
against the closed-form field they interpolate; the targets against their
definition on a Cartesian element with constant c^2 (where they vanish)."""
import numpy as np

from oracle import general, mlp
from paper_2105_01722_amd import inputs

NI, H, K = 64, 16, 9


def _theta(seed=0):
    rng = np.random.default_rng(seed)
    sz = sum(mlp.param_sizes(NI, H, K))
    return 0.3 * rng.standard_normal(sz)


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal((7, NI)), rng.standard_normal((7, K))
    th = _theta()
    _, g = mlp.loss_and_grad(th, x, y, NI, H, K)
    idx = rng.choice(th.size, 40, replace=False)
    for i in idx:
        e = np.zeros_like(th)
        e[i] = 1e-6
        lp, _ = mlp.loss_and_grad(th + e, x, y, NI, H, K)
        lm, _ = mlp.loss_and_grad(th - e, x, y, NI, H, K)
        fd = (lp - lm) / 2e-6
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


def test_adam_first_step():
    """First Adam step with bias correction moves every parameter by lr * sign(g)
    (m_hat = g, v_hat = g^2)."""
    g = np.array([0.5, -2.0, 1e-3])
    th, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(th, -0.01 * np.sign(g), rtol=1e-12)


def test_forward_shapes_and_relu():
    th = _theta(2)
    x = np.zeros((3, NI))
    out, (xx, z1, h1, z2, h2) = mlp.forward(th, x, NI, H, K)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th, NI, H, K)
    np.testing.assert_allclose(h1[0], np.maximum(b1, 0))
    assert out.shape == (3, K)


def test_coefficient_samples_interpolate_the_field():
    """The GD interpolant of a field that is a polynomial of degree <= p in each variable
    reproduces it exactly at the sample centres."""
    n, N, p = 2, 8, 3
    X, Y = inputs.node_coords(n, n, N)
    f = lambda x, y: 1.0 + 0.3 * x ** 3 - 0.2 * x * y ** 2 + 0.1 * y
    s = mlp.coefficient_samples(f(X, Y), N, p)
    c = (np.arange(8) + 0.5) / 8 * 0.5
    for ey in range(n):
        for ex in range(n):
            xs = ex * 0.5 + c[None, :]
            ys = ey * 0.5 + c[:, None]
            np.testing.assert_allclose(s[ey * n + ex], ((f(xs, ys) - 1) / 0.5).ravel(), atol=1e-12)


def test_targets_vanish_on_cartesian_constant():
    """With constant c^2 on a Cartesian element the plain preconditioner is exact, so the
    exact modal diagonal equals D and the targets are 0."""
    n, N, p = 2, 6, 3
    X, Y = inputs.node_coords(n, n, N)
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p), X, Y, np.full_like(X, 1.7))
    np.testing.assert_allclose(mlp.modal_targets(ops), 0.0, atol=1e-9)


def test_targets_small_but_nonzero_on_variable_coefficient():
    n, N, p = 2, 6, 3
    X, Y = inputs.node_coords(n, n, N)
    ops = general.GenOps(general.GenProblem(nx=n, ny=n, N=N, p=p), X, Y, inputs.c2_field(3, X, Y))
    o = mlp.modal_targets(ops)
    assert o.shape == (4, 48) and 1e-6 < np.abs(o).max() < 1.0
