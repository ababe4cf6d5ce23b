"""Workloads at their full size, in the launch configuration the benchmark
times, checked through properties that hold at any size: the output TT,
evaluated at random grid points, against the elementwise function of the
input TTs evaluated at the same points (a value computed one point at a time
from the definition of the result), the rank caps, and the error estimate.

* product of two random 3D Fourier fields (1024^3 grid, L = 30, d = 2, TT
  rank 128), tol 1e-8, rank cap 192, FP64, fixed sweeps;
* |psi|^2 psi of a 2D vortex-speckle field ((2^14)^2 grid, L = 28, TT rank
  512), rank cap 512, complex128 and complex64 contractions;
* one explicit Gross-Pitaevskii step of the same field (second differences
  by MPO, inputs of rank 1536, then ACI started from psi), against the
  Euler step evaluated from psi at each sample point and its four
  neighbours.

Bounds.  A cross interpolation reproduces the function exactly on its
pivots; between them the error of each two-site update is estimated by the
first rejected pivot.  The global error is at most the sum of the local ones
over the 2(L - 1) updates of a sweep, so samples must stay within
2 (L - 1) max_eps (times a factor two for the estimate itself being a
sample of the residual), relative to the largest value of the function."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")

SAMPLES = 4096


def cores_on(x, device):
    return [torch.from_numpy(np.ascontiguousarray(c)).to(device) for c in x]


def sampled_error(out_cores, f, points):
    y = W.tt_eval([c.cpu().numpy() for c in out_cores], points)
    return np.abs(y - f).max()


def test_fourier_product_full_size_sampled():
    dev = torch.device("cuda:0")
    u, v = W.fourier3d_pair(R=10, kmax=32, chi=128, seeds=(2001, 2002), device=dev)
    L = len(u)
    assert L == 30 and max(c.shape[2] for c in u) == 128
    S = aci.Session([cores_on(u, dev), cores_on(v, dev)], "product", 1e-8, 192, maxiter=12, seed=2003,
                    fixed_sweeps=True)
    st = S.sweep(12)
    cores, info = S.result()
    S.close()
    assert max(st["ranks"]) <= 192
    rng = np.random.default_rng(91)
    pts = rng.integers(0, 2, (SAMPLES, L))
    f = W.tt_eval(u, pts) * W.tt_eval(v, pts)
    scale = max(np.abs(f).max(), 1e-300)
    err = sampled_error(cores, f, pts)
    print(f"fourier product: sampled max err {err / scale:.3e} (relative), max eps {st['max_eps']:.3e}")
    assert np.isfinite(st["max_eps"])
    assert err <= 4 * (L - 1) * st["max_eps"] + 1e-12 * scale


@pytest.fixture(scope="module")
def gp_psi():
    return W.gp_field(R=14, chi=512, seed=5001, device=torch.device("cuda:0"), waves=16, kmax=256)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gross_pitaevskii_full_size_sampled(precision, gp_psi):
    dev = torch.device("cuda:0")
    psi = gp_psi
    L = len(psi)
    assert L == 28 and max(c.shape[2] for c in psi) == 512
    S = aci.Session([cores_on(psi, dev)], "abs2_mul", 1e-8, 512, maxiter=3, seed=2003, fixed_sweeps=True,
                    precision=precision, low_precision_sweeps=-1)
    st = S.sweep(3)
    cores, info = S.result()
    S.close()
    assert max(st["ranks"]) <= 512
    rng = np.random.default_rng(92)
    pts = rng.integers(0, 2, (SAMPLES, L))
    z = W.tt_eval(psi, pts)
    f = (z.real * z.real + z.imag * z.imag) * z
    scale = max(np.abs(f).max(), 1e-300)
    err = sampled_error(cores, f, pts)
    print(f"GP {precision}: sampled max err {err / scale:.3e} (relative), max eps {st['max_eps']:.3e}")
    assert err <= 4 * (L - 1) * st["max_eps"] + 1e-12 * scale


def quantics_neighbours(pts, R, ndim, axis, delta):
    """Quantics digits of the grid points one step along ``axis`` (periodic);
    site ndim*b + a holds bit R-1-b of axis a."""
    out = pts.copy()
    sites = [ndim * b + axis for b in range(R)]
    coord = np.zeros(pts.shape[0], dtype=np.int64)
    for b, s in enumerate(sites):
        coord |= pts[:, s].astype(np.int64) << (R - 1 - b)
    coord = (coord + delta) % (1 << R)
    for b, s in enumerate(sites):
        out[:, s] = (coord >> (R - 1 - b)) & 1
    return out


def test_gross_pitaevskii_step_full_size_sampled(gp_psi):
    dev = torch.device("cuda:0")
    psi = gp_psi
    R, ndim, L = 14, 2, len(psi)
    dt = 0.1 / 4.0 ** R
    c0, c_lap, c3 = 1.0, 0.5j * dt, -1j * dt
    cores, info = aci.cubic_step(cores_on(psi, dev), ndim, c0, c_lap, c3, 1e-8, 512, maxiter=3,
                                 fixed_sweeps=True)
    assert max(info.ranks) <= 512
    rng = np.random.default_rng(93)
    pts = rng.integers(0, 2, (SAMPLES, L))
    z = W.tt_eval(psi, pts)
    lap = 0.0
    for a in range(ndim):
        lap = lap + (W.tt_eval(psi, quantics_neighbours(pts, R, ndim, a, 1)) - 2 * z
                     + W.tt_eval(psi, quantics_neighbours(pts, R, ndim, a, -1))) * 4.0 ** R
    f = c0 * z + c_lap * lap + c3 * (z.real * z.real + z.imag * z.imag) * z
    scale = max(np.abs(f).max(), 1e-300)
    err = sampled_error(cores, f, pts)
    max_eps = max(info.eps)
    print(f"GP step: sampled max err {err / scale:.3e} (relative), max eps {max_eps:.3e}, "
          f"ranks <= {max(info.ranks)}")
    assert err <= 4 * (L - 1) * max_eps + 1e-12 * scale

