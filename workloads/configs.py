"""Named input recipes (the workloads the parity tests and the bench run).

* ``random_pair``   -- two random TTs, cores N(0, 1/chi), left-orthogonalised
                       (the random-TT experiment of section 3.3, here with
                       Gaussian cores so that the exact product has full rank
                       chi^2).
* ``fourier3d_pair``-- two random 3D Fourier fields with a k^-5/3 shell
                       spectrum on an interleaved quantics grid, compressed by
                       TT-SVD (3D analogue of the random Fourier series of
                       section 3.2).
* ``gp_field``      -- complex 2D vortex field for the |psi|^2 psi term.
* ``velocity_set``  -- three velocity components and their nine spectral
                       derivatives for the convective products u_j d_j u_k.
* ``random_init``   -- explicit initial guess Y_init with given ranks.
"""

from __future__ import annotations

import numpy as np

from .tt import random_tt, left_orthogonalise, tt_svd
from .fields import grid_to_quantics, fourier3d_full, gp_vortex_full


def random_pair(L=12, d=2, chi=8, seeds=(1001, 1002), dtype=np.float64):
    return tuple(left_orthogonalise(random_tt(L, d, chi, s, dtype=dtype)) for s in seeds)


def random_init(ranks, d, seed, dtype=np.float64):
    """Y_init with bond ranks ``ranks`` (length L+1, ends 1) and i.i.d. N(0,1)
    entries from PCG64(seed), site by site in C order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cores = []
    for s in range(len(ranks) - 1):
        shape = (ranks[s], d, ranks[s + 1])
        if np.issubdtype(np.dtype(dtype), np.complexfloating):
            c = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        else:
            c = rng.standard_normal(shape)
        cores.append(np.ascontiguousarray(c, dtype=dtype))
    return cores


def min_ranks(inputs, maxrank):
    """Bond ranks min_n r^n_l capped by maxrank (the default Y_init ranks)."""
    L = len(inputs[0])
    r = [1]
    for s in range(L - 1):
        r.append(min(min(x[s].shape[2] for x in inputs), maxrank))
    r.append(1)
    return r


def _compress(grid, R, ndim, chi, device):
    q = grid_to_quantics(grid, R, ndim)
    if device is None:
        flat = np.ascontiguousarray(q).reshape(-1)
        return tt_svd(flat, 2, chi, rtol=1e-14)
    return tt_svd(q, 2, chi, rtol=1e-14, method="gram")


def fourier3d_pair(R=10, kmax=32, chi=128, seeds=(2001, 2002), device=None, progress=None):
    out = []
    for s in seeds:
        g = fourier3d_full(R, kmax, s, device=device)
        if progress:
            progress(f"field seed {s} sampled")
        out.append(_compress(g, R, 3, chi, device))
        del g
        if progress:
            progress(f"field seed {s} compressed")
    return tuple(out)


def fourier3d_field(R=10, kmax=32, chi=128, seed=2001, device=None):
    """One random 3D Fourier field of the main recipe compressed to rank chi."""
    g = fourier3d_full(R, kmax, seed, device=device)
    return _compress(g, R, 3, chi, device)


def gp_field(R=14, chi=512, seed=5001, device=None, width_scale=1.0, waves=0, kmax=48):
    g = gp_vortex_full(R, seed, device=device, width_scale=width_scale, waves=waves, kmax=kmax)
    return _compress(g, R, 2, chi, device)


def velocity_set(R=10, kmax=32, seeds=(3001, 3002, 3003),
                 chi_u=(64, 96, 128), chi_du=(128, 192, 256), device=None, deriv="central"):
    """u_j compressed to chi_u[j]; d_j u_k (periodic central difference of
    the same Fourier field on the grid, or its spectral derivative) compressed
    to chi_du[(j + k) % 3].  Returns (u, du) with du[j][k] the TT of
    d u_k / d x_j."""
    u = []
    for j, s in enumerate(seeds):
        g = fourier3d_full(R, kmax, s, device=device)
        u.append(_compress(g, R, 3, chi_u[j], device))
        del g
    du = [[None] * 3 for _ in range(3)]
    for j in range(3):
        for k, s in enumerate(seeds):
            g = fourier3d_full(R, kmax, s, device=device, deriv_axis=j, deriv=deriv)
            du[j][k] = _compress(g, R, 3, chi_du[(j + k) % 3], device)
            del g
    return u, du
