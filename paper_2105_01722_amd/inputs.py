"""Seeded synthetic inputs shared by the HIP path's callers and by the tests.

This module holds no part of the method: it only produces nodal sample arrays
(initial data, coefficient fields, node coordinates) with numpy's PCG64
generator.  The same arrays are handed to the HIP library and to the CPU
oracle.

Layout of every nodal array: [ny, nx, N+1 (iy), N+1 (ix)], element e = ey*nx + ex,
node (ix, iy) of element e at flat offset e*(N+1)^2 + iy*(N+1) + ix.  Nodes on
element faces are duplicated (one copy per element).

Workloads (all periodic on [0,1]^2):
  * standing wave  u0 = sin(2 pi x) sin(2 pi y), v0 = 0; exact
    u = u0 cos(2 sqrt(2) pi c t).
  * Fourier superposition: for m = 1..8, k_m uniform on {k in Z^2 \\ 0 : |k| <= 16},
    a_m ~ N(0,1)/|k_m|^2, theta_m ~ U[0, 2 pi); u0 = sum a_m cos(2 pi k_m.x + theta_m),
    v0 = 0; exact u = sum a_m cos(2 pi |k_m| c t) cos(2 pi k_m.x + theta_m).
  * smooth periodic Gaussian random field g (length scale 0.1): a random cosine
    series over wave vectors 0 < |k| <= 10 (one half-plane) with amplitudes
    N(0, exp(-2 pi^2 l^2 |k|^2)), normalised to unit variance, clipped to [-0.9, 0.9];
    c^2 = 1 + 0.5 g.
  * mapped mesh: X = x + eps s, Y = y + eps s with s = sin(2 pi x) sin(2 pi y),
    eps = 0.05 (the identity on the boundary of the unit square).
"""
import numpy as np


def node_coords(nx, ny, N, Lx=1.0, Ly=1.0, x0=0.0, y0=0.0):
    """Cartesian node coordinates X, Y ([ny, nx, N+1, N+1]).

    Coordinates are computed from the global node index so that the two copies of a
    face node (one per element) are bitwise identical.
    """
    n1 = N + 1
    gx = np.arange(nx)[:, None] * N + np.arange(n1)[None, :]          # [nx, n1]
    gy = np.arange(ny)[:, None] * N + np.arange(n1)[None, :]          # [ny, n1]
    xs = x0 + gx * (Lx / (nx * N))
    ys = y0 + gy * (Ly / (ny * N))
    X = np.broadcast_to(xs[None, :, None, :], (ny, nx, n1, n1)).copy()
    Y = np.broadcast_to(ys[:, None, :, None], (ny, nx, n1, n1)).copy()
    return X, Y


def standing_wave(X, Y):
    return np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)


def fourier_modes(seed, n_modes=8, kmax=16):
    """Draw (kx, ky, a, theta) for `n_modes` modes, |k| <= kmax, k != 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = [(i, j) for i in range(-kmax, kmax + 1) for j in range(-kmax, kmax + 1)
          if 0 < i * i + j * j <= kmax * kmax]
    out = []
    for _ in range(n_modes):
        kx, ky = ks[int(rng.integers(len(ks)))]
        k2 = float(kx * kx + ky * ky)
        a = float(rng.standard_normal()) / k2
        th = float(rng.uniform(0.0, 2 * np.pi))
        out.append((kx, ky, a, th))
    return out


def fourier_field(modes, X, Y, t=0.0, c=1.0):
    """sum_m a_m cos(2 pi |k_m| c t) cos(2 pi k_m . x + theta_m)."""
    u = np.zeros(np.broadcast(X, Y).shape)
    for kx, ky, a, th in modes:
        kn = np.hypot(kx, ky)
        u += a * np.cos(2 * np.pi * kn * c * t) * np.cos(2 * np.pi * (kx * X + ky * Y) + th)
    return u


def grf(seed, X, Y, ell=0.1, kmax=10, clip=0.9):
    """Clipped smooth periodic Gaussian random field sampled at (X, Y)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = [(i, j) for i in range(-kmax, kmax + 1) for j in range(0, kmax + 1)
          if 0 < i * i + j * j <= kmax * kmax and (j > 0 or i > 0)]
    var = np.array([np.exp(-2 * np.pi ** 2 * ell ** 2 * (i * i + j * j)) for i, j in ks])
    amp = rng.standard_normal(len(ks)) * np.sqrt(var)
    th = rng.uniform(0.0, 2 * np.pi, len(ks))
    Z = np.sqrt(0.5 * var.sum())
    g = _cos_series(ks, amp, th, X, Y)
    return np.clip(g / Z, -clip, clip)


def _separable(X, Y):
    """True when X, Y are [ny, nx, n1, n1] arrays with X a function of (ex, ix) only and
    Y of (ey, iy) only (Cartesian node arrays)."""
    X, Y = np.asarray(X), np.asarray(Y)
    if X.ndim != 4 or X.shape != Y.shape:
        return False
    return (np.array_equal(X, np.broadcast_to(X[:1, :, :1, :], X.shape))
            and np.array_equal(Y, np.broadcast_to(Y[:, :1, :, :1], Y.shape)))


def _cos_series(ks, amp, th, X, Y):
    """sum_k amp_k cos(2 pi (i_k X + j_k Y) + th_k).  On Cartesian node arrays the sum is
    evaluated as one complex matrix product over the distinct x and y values."""
    if _separable(X, Y):
        ny, nx, n1, _ = X.shape
        xs = X[0, :, 0, :].ravel()                       # (ex, ix)
        ys = Y[:, 0, :, 0].ravel()                       # (ey, iy)
        ki = np.array([k[0] for k in ks], dtype=np.float64)
        kj = np.array([k[1] for k in ks], dtype=np.float64)
        A = (amp * np.exp(1j * th))[None, :] * np.exp(2j * np.pi * ys[:, None] * kj[None, :])
        B = np.exp(2j * np.pi * ki[:, None] * xs[None, :])
        g = (A @ B).real.reshape(ny, n1, nx, n1)         # [ey, iy, ex, ix]
        return np.ascontiguousarray(g.transpose(0, 2, 1, 3))
    g = np.zeros(np.broadcast(X, Y).shape)
    for (i, j), a, t in zip(ks, amp, th):
        g += a * np.cos(2 * np.pi * (i * X + j * Y) + t)
    return g


def c2_field(seed, X, Y):
    """c^2 = 1 + 0.5 g with g the clipped field above (values in [0.55, 1.45])."""
    return 1.0 + 0.5 * grf(seed, X, Y)


def mapped_coords(X, Y, eps=0.05):
    s = np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    return X + eps * s, Y + eps * s


def batch_specs(seed=4, n_prob=64):
    """Independent problems of uneven size and degree: n ~ U{16..128} elements per
    direction, N ~ U{8, 12, 16}, p ~ U{3, 5, 7}, half of them (alternating) with a variable
    coefficient on the mapped mesh.  Returns dicts (n, N, p, variable, grf_seed, mode_seed);
    problem i uses coefficient seed 1000 + i and initial-data seed 2000 + i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_prob):
        n = int(rng.integers(16, 129))
        N = int(rng.choice([8, 12, 16]))
        p = int(rng.choice([3, 5, 7]))
        out.append(dict(n=n, N=N, p=p, variable=(i % 2 == 1), grf_seed=1000 + i,
                        mode_seed=2000 + i))
    return out


def cfl_dt(N, n, cfl=0.5, L=1.0):
    """dt = CFL * h with h = L / (n N) the cell width."""
    return cfl * L / (n * N)


# ---- box elements in 3D ----------------------------------------------------------------
def node_coords3(nx, ny, nz, N, Lx=1.0, Ly=1.0, Lz=1.0, x0=0.0, y0=0.0, z0=0.0):
    """Cartesian node coordinates of a 3D grid, each [nz, ny, nx, N+1 (iz), N+1 (iy),
    N+1 (ix)], from the global node index (face copies bitwise equal)."""
    n1 = N + 1
    gx = (np.arange(nx)[:, None] * N + np.arange(n1)[None, :]) * (Lx / (nx * N)) + x0
    gy = (np.arange(ny)[:, None] * N + np.arange(n1)[None, :]) * (Ly / (ny * N)) + y0
    gz = (np.arange(nz)[:, None] * N + np.arange(n1)[None, :]) * (Lz / (nz * N)) + z0
    shp = (nz, ny, nx, n1, n1, n1)
    X = np.broadcast_to(gx[None, None, :, None, None, :], shp)
    Y = np.broadcast_to(gy[None, :, None, None, :, None], shp)
    Z = np.broadcast_to(gz[:, None, None, :, None, None], shp)
    return X, Y, Z


def fourier_modes3(seed, n_modes=8, kmax=8):
    """(kx, ky, kz, a, theta) for n_modes modes, |k| <= kmax, k != 0, a ~ N(0,1)/|k|^2,
    theta ~ U[0, 2 pi) (the 3D analogue of fourier_modes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = range(-kmax, kmax + 1)
    ks = [(i, j, k) for i in r for j in r for k in r if 0 < i * i + j * j + k * k <= kmax * kmax]
    out = []
    for _ in range(n_modes):
        kx, ky, kz = ks[int(rng.integers(len(ks)))]
        a = float(rng.standard_normal()) / float(kx * kx + ky * ky + kz * kz)
        th = float(rng.uniform(0.0, 2 * np.pi))
        out.append((kx, ky, kz, a, th))
    return out


def fourier_field3(modes, X, Y, Z, t=0.0, c=1.0, deriv=False):
    """sum_m a_m cos(2 pi |k_m| c t) cos(2 pi k_m . x + theta_m) on node arrays of
    node_coords3 (deriv: its time derivative).  Evaluated per element row through the
    separable factors, so that large grids need no full-size temporaries per mode."""
    nz, ny, nx, n1 = X.shape[0], X.shape[1], X.shape[2], X.shape[3]
    xs = np.asarray(X[0, 0, :, 0, 0, :])      # [nx, n1]
    ys = np.asarray(Y[0, :, 0, 0, :, 0])      # [ny, n1]
    zs = np.asarray(Z[:, 0, 0, :, 0, 0])      # [nz, n1]
    out = np.zeros((nz, ny, nx, n1, n1, n1))
    for kx, ky, kz, a, th in modes:
        w = 2 * np.pi * np.sqrt(kx * kx + ky * ky + kz * kz) * c
        amp = -a * w * np.sin(w * t) if deriv else a * np.cos(w * t)
        ex = np.exp(2j * np.pi * kx * xs)     # [nx, n1]
        ey = np.exp(2j * np.pi * ky * ys)
        ez = np.exp(2j * np.pi * kz * zs) * np.exp(1j * th)
        # [nz, ny, nx, iz, iy, ix]
        out += amp * np.real(ez[:, None, None, :, None, None] * ey[None, :, None, None, :, None]
                             * ex[None, None, :, None, None, :])
    return out
