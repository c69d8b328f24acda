"""1D Galerkin-difference (GD) space on one element -- FP64 oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper: Sec. 2.1 (the generating function Phi_p, eq. GD_basis_lagrange, the
nodal form eq. GD_basis_nodalformula), Sec. 2.1.1 (extrapolation closure and the
p = 3 worked example), Sec. 3.1 (1D mass and stiffness, bandwidth p) and
Sec. 3.2 (surface vectors phi(L), phi(R), phi'(L), phi'(R)).

Reading used here (the paper states the closure only for p = 3; for larger p it
extrapolates to the accuracy of the interior formulas): ghost values are
the degree-p polynomial through nodes 0..p (N-p..N on the right).  On a cell
whose interior stencil reaches a ghost node every stencil value then lies on
that polynomial, so the cell interpolant *is* that polynomial.  Hence on cell k
(between nodes k and k+1, unit spacing) the function is the degree-p Lagrange
interpolant on the window {s_k, ..., s_k + p}, s_k = clamp(k - (p-1)/2, 0, N-p).
Interior cells get the centred window of eq. GD_basis_lagrange.  N >= p keeps
the two closures apart.

Coordinates: t in [0, N] with unit node spacing; physical x = x_L + h t,
h = H / N.  The unit-spacing matrices are M_hat, S_hat, d_hat; physical ones are
M = h M_hat, S = S_hat / h, d = d_hat / h.
"""
import numpy as np


def check_degree(N, p):
    """p odd and N >= p (Sec. 2: odd degree; closure needs N >= p)."""
    if p < 1 or p % 2 == 0:
        raise ValueError("GD degree p must be odd and >= 1, got %r" % (p,))
    if N < p:
        raise ValueError("need N >= p (cells per element >= degree), got N=%r p=%r" % (N, p))


def window_start(k, N, p):
    """First node of the p+1 point stencil used on cell k (closure reading above)."""
    return min(max(k - (p - 1) // 2, 0), N - p)


def lagrange_values(nodes, t):
    """Values of the Lagrange basis on `nodes` at points t: array [len(t), len(nodes)]."""
    nodes = np.asarray(nodes, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    L = np.ones((t.size, nodes.size))
    for a in range(nodes.size):
        for b in range(nodes.size):
            if a != b:
                L[:, a] *= (t - nodes[b]) / (nodes[a] - nodes[b])
    return L


def lagrange_derivs(nodes, t):
    """First derivatives of the Lagrange basis on `nodes` at t: [len(t), len(nodes)].

    Product rule: l_a'(t) = sum_{b != a} 1/(x_a - x_b) prod_{c != a, b} (t - x_c)/(x_a - x_c).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = nodes.size
    D = np.zeros((t.size, n))
    for a in range(n):
        for b in range(n):
            if b == a:
                continue
            term = np.full(t.size, 1.0 / (nodes[a] - nodes[b]))
            for c in range(n):
                if c != a and c != b:
                    term *= (t - nodes[c]) / (nodes[a] - nodes[c])
            D[:, a] += term
    return D


def basis_on_cell(k, N, p, t):
    """All N+1 GD basis functions (values and t-derivatives) at points t in cell k.

    Returns (phi, dphi), each [len(t), N+1]; only the window columns are non-zero.
    Follows eq. GD_basis_nodalformula with the extrapolation closure.
    """
    s = window_start(k, N, p)
    w = np.arange(s, s + p + 1)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    phi = np.zeros((t.size, N + 1))
    dphi = np.zeros((t.size, N + 1))
    phi[:, w] = lagrange_values(w, t)
    dphi[:, w] = lagrange_derivs(w, t)
    return phi, dphi


def basis_eval(N, p, t):
    """Evaluate the whole basis at arbitrary t in [0, N] (cell chosen by floor(t))."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    k = np.clip(np.floor(t).astype(int), 0, N - 1)
    phi = np.zeros((t.size, N + 1))
    dphi = np.zeros((t.size, N + 1))
    for kk in np.unique(k):
        sel = k == kk
        a, b = basis_on_cell(int(kk), N, p, t[sel])
        phi[sel] = a
        dphi[sel] = b
    return phi, dphi


def gauss_legendre(npts):
    """Gauss-Legendre nodes/weights on [0, 1] (library routine on [-1, 1], mapped)."""
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (x + 1.0), 0.5 * w


def matrices_unit(N, p):
    """Unit-spacing 1D mass M_hat and stiffness S_hat, each (N+1) x (N+1).

    M_hat_ij = sum_k int_k^{k+1} phi_i phi_j dt and S_hat_ij = sum_k int phi_i' phi_j' dt
    (Sec. 3.1: M_{j,kl} and S_{j,kl}).  A (p+1)-point Gauss rule per cell is exact for
    these degree-2p integrands.
    """
    check_degree(N, p)
    xg, wg = gauss_legendre(p + 1)
    M = np.zeros((N + 1, N + 1))
    S = np.zeros((N + 1, N + 1))
    for k in range(N):
        phi, dphi = basis_on_cell(k, N, p, k + xg)
        M += phi.T @ (wg[:, None] * phi)
        S += dphi.T @ (wg[:, None] * dphi)
    return M, S


def face_vectors_unit(N, p):
    """d_hat_L = phi_i'(0) and d_hat_R = phi_i'(N) (the non-zeros of D-tilde, Sec. 3.2).

    phi_i(0) = delta_{i0} and phi_i(N) = delta_{iN} because the basis is interpolatory.
    """
    _, dL = basis_on_cell(0, N, p, [0.0])
    _, dR = basis_on_cell(N - 1, N, p, [float(N)])
    return dL[0].copy(), dR[0].copy()


def element_1d(N, p, H):
    """Physical 1D data of an element of width H: (M, S, dL, dR), h = H / N."""
    Mh, Sh = matrices_unit(N, p)
    dL, dR = face_vectors_unit(N, p)
    h = H / N
    return h * Mh, Sh / h, dL / h, dR / h
