"""Sampled functions on quantics grids (section 3 of the paper).

Quantics encoding (Eq. quanticsrep): a grid coordinate ``x`` in
``[x_min, x_max)`` with ``2^R`` points is written as
``(x - x_min)/(x_max - x_min) = sum_b 2^{-b} sigma_b`` with sigma_1 the most
significant bit.  For several axes the bits are interleaved level by level:
site ``ndim*(b-1) + a`` holds bit b of axis a.

Dense fields are produced as numpy arrays (or torch tensors when a torch
device is given, for the 2^28--2^30 point grids) and compressed to TTs by
``workloads.tt.tt_svd``.
"""

from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------- quantics
def quantics_points_1d(R, x_min=0.0, x_max=1.0):
    return x_min + (x_max - x_min) * np.arange(2 ** R, dtype=np.float64) / 2 ** R


def grid_to_quantics(F, R, ndim):
    """Dense grid array of shape ``(2^R,)*ndim`` -> interleaved quantics order.

    numpy input: a tensor of shape ``(2,)*(ndim*R)`` (a transposed view).
    torch input: a flat contiguous tensor of 2^(ndim R) entries in C order
    over the sites (built by a chunked gather, since torch tensors are
    limited to 16 dimensions)."""
    if isinstance(F, np.ndarray):
        t = F.reshape((2,) * (ndim * R))
        perm = [a * R + b for b in range(R) for a in range(ndim)]
        return np.transpose(t, perm)
    import torch
    flat = F.reshape(-1)
    total = flat.numel()
    out = torch.empty_like(flat)
    n = 2 ** R
    nbits = ndim * R
    # bit t of the quantics index (t = 0 least significant) is site
    # s = nbits - 1 - t, i.e. bit R-1-b of axis a with s = ndim*b + a; its
    # weight in the C-order grid index is 2^(R-1-b) * n^(ndim-1-a).  The
    # grid index is linear in these bits, so two tables over the low and the
    # high half of the bits give it with one add.
    h = nbits // 2
    weights = []
    for t in range(nbits):
        s_ = nbits - 1 - t
        a, b = s_ % ndim, s_ // ndim
        weights.append((2 ** (R - 1 - b)) * n ** (ndim - 1 - a))

    def table(lo_bit, nb):
        v = np.zeros(2 ** nb, dtype=np.int64)
        for t in range(nb):
            v[(np.arange(2 ** nb) >> t) & 1 == 1] += weights[lo_bit + t]
        return torch.from_numpy(v).to(flat.device)

    t_lo = table(0, h)
    t_hi = table(h, nbits - h)
    chunk = 1 << 26
    for start in range(0, total, chunk):
        q = torch.arange(start, min(start + chunk, total), device=flat.device, dtype=torch.int64)
        src = t_hi[q >> h] + t_lo[q & ((1 << h) - 1)]
        out[start:start + q.numel()] = flat[src]
        del q, src
    return out


def quantics_to_grid(T, R, ndim):
    """Inverse of ``grid_to_quantics``."""
    perm = [a * R + b for b in range(R) for a in range(ndim)]
    inv = np.argsort(perm)
    t = np.transpose(np.asarray(T).reshape((2,) * (ndim * R)), inv)
    return t.reshape((2 ** R,) * ndim)


def _backend(device):
    if device is None:
        return np, None
    import torch
    return torch, torch.device(device)


# ---------------------------------------------------------------- Gaussians
def gaussian_pair_full(L, w=0.15, delta=0.4):
    """g_plus, g_minus of Eq. (gaussians) sampled on the quantics grid of
    [-0.5, 0.5) with L bits, plus the exact product
    exp(-x^2/w^2) * exp(-delta^2/(4 w^2))."""
    x = quantics_points_1d(L, -0.5, 0.5)
    gp = np.exp(-((x + delta / 2) ** 2) / (2 * w * w))
    gm = np.exp(-((x - delta / 2) ** 2) / (2 * w * w))
    h = np.exp(-(x * x) / (w * w)) * np.exp(-(delta * delta) / (4 * w * w))
    return gp, gm, h


# --------------------------------------------------- 1D random Fourier series
def fourier1d_coeffs(K, seed):
    """K+1 complex coefficients with Re, Im ~ U[0,1], normalised to unit
    2-norm (Eq. fourierseries)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(0.0, 1.0, K + 1) + 1j * rng.uniform(0.0, 1.0, K + 1)
    return c / np.linalg.norm(c)


def fourier1d_full(coeffs, L):
    """g(x) = sum_k c_k exp(i k x) on the quantics grid of [0, 1)."""
    x = quantics_points_1d(L, 0.0, 1.0)
    k = np.arange(len(coeffs))
    # sum over modes in blocks to bound memory
    out = np.zeros(x.shape, dtype=np.complex128)
    for k0 in range(0, len(coeffs), 64):
        kk = k[k0:k0 + 64]
        out += np.exp(1j * np.outer(x, kk)) @ coeffs[k0:k0 + 64]
    return out


def fourier1d_product_coeffs(c1, c2):
    """Coefficients of the product series: h_q = sum_k c1_k c2_{q-k}
    (the convolution written in Eq. fouriermultiplication; the printed
    half-integer index form is read as this convolution)."""
    return np.convolve(c1, c2)


# ------------------------------------------------- 3D random Fourier fields
def fourier3d_modes(kmax, seed, slope=-11.0 / 6.0):
    """Integer wave vectors 0 < |k| <= kmax in a half space (one of each +/-k
    pair), amplitude |k|^slope, phases U[0, 2 pi) drawn in lexicographic k
    order from PCG64(seed)."""
    r = np.arange(-kmax, kmax + 1)
    k1, k2, k3 = np.meshgrid(r, r, r, indexing="ij")
    k = np.stack([k1.ravel(), k2.ravel(), k3.ravel()], axis=1)
    n2 = (k * k).sum(1)
    half = (k[:, 2] > 0) | ((k[:, 2] == 0) & ((k[:, 1] > 0) | ((k[:, 1] == 0) & (k[:, 0] > 0))))
    sel = half & (n2 > 0) & (n2 <= kmax * kmax)
    k = k[sel]
    amp = np.sqrt((k * k).sum(1).astype(np.float64)) ** slope
    rng = np.random.Generator(np.random.PCG64(seed))
    phase = rng.uniform(0.0, 2 * np.pi, len(k))
    return k, amp, phase


def fourier3d_full(R, kmax, seed, device=None, deriv_axis=None, deriv="spectral"):
    """u(x) = sum_k A_k cos(2 pi k.x + phi_k) on the (2^R)^3 grid of [0,1)^3,
    normalised to RMS 1 (over the grid the modes are orthogonal, so the RMS is
    sqrt(sum A_k^2 / 2)).  With ``deriv_axis=j`` returns d u / d x_j under the
    same normalisation factor: ``deriv="spectral"`` the exact derivative,
    ``"central"`` the periodic central difference (u(x + h e_j) -
    u(x - h e_j)) / 2h on the grid (h = 2^-R), which multiplies each mode by
    i sin(2 pi k_j h) / h.  Computed as three separable small-DFT sums.
    Returns a (2^R)^3 array (numpy, or a torch tensor on ``device``)."""
    k, amp, phase = fourier3d_modes(kmax, seed)
    norm = np.sqrt((amp * amp).sum() / 2.0)
    coef = amp * np.exp(1j * phase) / norm             # u = Re sum coef e^{2 pi i k.x}
    if deriv_axis is not None:
        if deriv == "spectral":
            coef = coef * (2j * np.pi * k[:, deriv_axis])
        elif deriv == "central":
            h = 2.0 ** -R
            coef = coef * (1j * np.sin(2 * np.pi * k[:, deriv_axis] * h) / h)
        else:
            raise ValueError(f"unknown derivative {deriv!r}")
    nk = 2 * kmax + 1
    C = np.zeros((nk, nk, nk), dtype=np.complex128)
    np.add.at(C, (k[:, 0] + kmax, k[:, 1] + kmax, k[:, 2] + kmax), coef)
    n = 2 ** R
    idx = np.arange(n)
    kk = np.arange(-kmax, kmax + 1)
    E = np.exp(2j * np.pi * np.outer(idx, kk) / n)       # n x nk
    xp, dev = _backend(device)
    if dev is None:
        T1 = np.einsum("abc,zc->abz", C, E)               # nk x nk x n
        T2 = np.einsum("yb,abz->ayz", E, T1)              # nk x n x n
        T2 = T2.reshape(nk, n * n)
        U = E.real @ T2.real - E.imag @ T2.imag          # n x n^2
        return U.reshape(n, n, n)
    torch = xp
    Ct = torch.from_numpy(C).to(dev)
    Et = torch.from_numpy(E).to(dev)
    T1 = torch.einsum("abc,zc->abz", Ct, Et)
    T2 = torch.einsum("yb,abz->ayz", Et, T1).reshape(nk, n * n)
    U = Et.real @ T2.real - Et.imag @ T2.imag
    del T1, T2
    return U.reshape(n, n, n)


# ------------------------------------------- Gross-Pitaevskii vortex field
def gp_vortex_params(seed, modes=32):
    rng = np.random.Generator(np.random.PCG64(seed))
    a = (rng.standard_normal(modes) + 1j * rng.standard_normal(modes)) / np.sqrt(2.0)
    centres = rng.uniform(0.15, 0.85, (modes, 2))
    widths = rng.uniform(0.03, 0.10, modes)
    signs = np.where(rng.uniform(0.0, 1.0, modes) < 0.5, -1.0, 1.0)
    return a, centres, widths, signs


def gp_wave_params(seed, modes=32, waves=8, kmax=48):
    """Random plane-wave content of each mode: integer wavevectors with
    components in [-kmax, kmax] and complex normal amplitudes."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    k = rng.integers(-kmax, kmax + 1, (modes, waves, 2))
    b = (rng.standard_normal((modes, waves)) + 1j * rng.standard_normal((modes, waves))) / np.sqrt(2.0 * waves)
    return k, b


def gp_vortex_full(R, seed, modes=32, device=None, width_scale=1.0, waves=0, kmax=48):
    """psi(x, y) = sum_m a_m ((x-x_m) + i s_m (y-y_m))/w_m
    exp(-((x-x_m)^2 + (y-y_m)^2)/(2 w_m^2)) S_m(x, y) on the (2^R)^2 grid of
    [0,1)^2, normalised to max |psi| = 1 over the grid.  S_m = 1 when
    ``waves`` is 0; otherwise S_m = sum_j b_mj exp(2 pi i k_mj . (x, y)) is a
    random superposition of ``waves`` plane waves (|k_j| <= kmax per axis),
    which fills every mode with phase singularities (a speckle of vortices)
    and raises the quantics ranks.  Every term is separable in x and y, so
    the waves > 0 field is assembled as one product X Y^T of n x (2 modes
    waves) factors."""
    a, c, w, s = gp_vortex_params(seed, modes)
    w = w * width_scale
    n = 2 ** R
    xp, dev = _backend(device)
    if waves > 0:
        k, b = gp_wave_params(seed, modes, waves, kmax)
        x = np.arange(n, dtype=np.float64) / n
        X = np.empty((n, modes, waves, 2), dtype=np.complex128)
        Y = np.empty((n, modes, waves, 2), dtype=np.complex128)
        for m in range(modes):
            dx, dy = x - c[m, 0], x - c[m, 1]
            gx = np.exp(-dx * dx / (2 * w[m] ** 2))
            gy = np.exp(-dy * dy / (2 * w[m] ** 2))
            ex = np.exp(2j * np.pi * np.outer(x, k[m, :, 0]))     # n x waves
            ey = np.exp(2j * np.pi * np.outer(x, k[m, :, 1]))
            coef = a[m] * b[m] / w[m]
            X[:, m, :, 0] = (dx * gx)[:, None] * ex * coef
            Y[:, m, :, 0] = gy[:, None] * ey
            X[:, m, :, 1] = gx[:, None] * ex * (1j * s[m]) * coef
            Y[:, m, :, 1] = (dy * gy)[:, None] * ey
        X = X.reshape(n, -1)
        Y = Y.reshape(n, -1)
        if dev is None:
            psi = X @ Y.T
            return psi / np.abs(psi).max()
        torch = xp
        psi = torch.from_numpy(X).to(dev) @ torch.from_numpy(np.ascontiguousarray(Y.T)).to(dev)
        return psi / psi.abs().max()
    if dev is None:
        x = np.arange(n, dtype=np.float64) / n
        psi = np.zeros((n, n), dtype=np.complex128)
        for m in range(modes):
            dx = (x - c[m, 0])[:, None]
            dy = (x - c[m, 1])[None, :]
            g = np.exp(-(dx * dx + dy * dy) / (2 * w[m] ** 2))
            psi += a[m] * ((dx + 1j * s[m] * dy) / w[m]) * g
        return psi / np.abs(psi).max()
    torch = xp
    x = torch.arange(n, dtype=torch.float64, device=dev) / n
    psi = torch.zeros((n, n), dtype=torch.complex128, device=dev)
    for m in range(modes):
        dx = (x - float(c[m, 0]))[:, None]
        dy = (x - float(c[m, 1]))[None, :]
        g = torch.exp(-(dx * dx + dy * dy) / (2 * float(w[m]) ** 2))
        psi += complex(a[m]) * ((dx + 1j * float(s[m]) * dy) / float(w[m])) * g
    return psi / psi.abs().max()
