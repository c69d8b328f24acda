"""FP64 reference of the learned preconditioner correction (not in the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A multilayer perceptron 64 -> H -> H -> K with ReLU activations maps the standardised
coefficient samples of one element, (c^2 - 1) / 0.5 at the centres of an 8 x 8
subdivision of the reference square, to K = (N+1)^2 - 1 log-multipliers o of the
diagonal D of the tensor-product preconditioner of the S_hat solve (every modal
entry except (0, 0)): D_k <- D_k exp(o_k).

Training target (supervised): o*_k = log(d_k / D_k), d = diag(Psi_2^T S_hat Psi_2), the
exact modal diagonal of the element operator in the reference eigenbasis; loss =
mean squared error over the minibatch and the K outputs; Adam (Kingma and Ba 2015)
with the textbook bias corrections.

Parameter layout (flat, float): W1 [H][64], b1 [H], W2 [H][H], b2 [H], W3 [K][H], b3 [K].
"""
import numpy as np

from . import gd1d, pcg


def param_sizes(n_in, hidden, n_out):
    return [hidden * n_in, hidden, hidden * hidden, hidden, n_out * hidden, n_out]


def unpack(theta, n_in, hidden, n_out):
    sz = param_sizes(n_in, hidden, n_out)
    off = np.cumsum([0] + sz)
    W1 = theta[off[0]:off[1]].reshape(hidden, n_in)
    b1 = theta[off[1]:off[2]]
    W2 = theta[off[2]:off[3]].reshape(hidden, hidden)
    b2 = theta[off[3]:off[4]]
    W3 = theta[off[4]:off[5]].reshape(n_out, hidden)
    b3 = theta[off[5]:off[6]]
    return W1, b1, W2, b2, W3, b3


def forward(theta, x, n_in, hidden, n_out):
    """Returns the output [B, K] and the cached pre-activations."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64), n_in, hidden, n_out)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ W3.T + b3
    return out, (x, z1, h1, z2, h2)


def loss_and_grad(theta, x, y, n_in, hidden, n_out):
    """MSE loss mean((out - y)^2) over B*K entries and its gradient (backpropagation)."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64), n_in, hidden, n_out)
    out, (x, z1, h1, z2, h2) = forward(theta, x, n_in, hidden, n_out)
    y = np.asarray(y, dtype=np.float64)
    B = x.shape[0]
    diff = out - y
    loss = float(np.mean(diff ** 2))
    dout = 2.0 * diff / (B * n_out)
    gW3 = dout.T @ h2
    gb3 = dout.sum(axis=0)
    dh2 = dout @ W3
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step count t >= 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def coefficient_samples(c2_nodal, N, p, ns=8):
    """(c^2 - 1)/0.5 of the GD interpolant at the centres of an ns x ns subdivision of each
    element: [n_el, ns*ns] (index j*ns + i for centre ((i+1/2)/ns, (j+1/2)/ns))."""
    t = (np.arange(ns) + 0.5) / ns * N
    B, _ = gd1d.basis_eval(N, p, t)                          # [ns, n1]
    ny, nx, n1, _ = c2_nodal.shape
    vals = np.einsum("sj,ri,eji->esr", B, B, c2_nodal.reshape(ny * nx, n1, n1))
    return ((vals - 1.0) / 0.5).reshape(ny * nx, ns * ns)


def modal_targets(ops):
    """o*_k = log(d_k / D_k) for every element (k over the (N+1)^2 - 1 modes after (0, 0))."""
    P = pcg.TensorPreconditioner(ops)
    P2 = np.kron(P.Psi, P.Psi)                               # [(iy,ix), (ky,kx)]
    d = np.einsum("ik,eij,jk->ek", P2, ops.Shat, P2)
    D = P.DS.reshape(d.shape)
    return np.log(d / D)[:, 1:]
