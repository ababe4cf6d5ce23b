"""TT operators on quantics grids and one explicit time step of a cubic
nonlinear equation, the use the outlook (Sec. 4) names for ACI.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A time step of a nonlinear PDE in tensor-train form consists of contractions
with TT operators (MPOs) of small, constant bond dimension -- here periodic
finite-difference stencils -- and an elementwise nonlinearity, which ACI
evaluates.  For

    dpsi/dt = k_lap Laplacian(psi) + k_lin psi + k_cub |psi|^2 psi

one explicit Euler step is the elementwise map

    y = c0 psi + c_lap sum_a D_a psi + c3 |psi|^2 psi,
    c0 = 1 + dt k_lin, c_lap = dt k_lap, c3 = dt k_cub,

of the N = 1 + ndim TTs (psi, D_1 psi, ..., D_ndim psi), with D_a the
second-difference operator along axis a.  The D_a psi are exact MPO-TT
contractions (bond ranks multiplied by the MPO's), and ACI is started from
psi itself (Y_init = psi, the warm start of section 2.6).

Grid convention: a periodic box [0,1)^ndim with 2^R points per axis,
spacing h = 2^-R; quantics sites interleave the bits level by level, site
``ndim*b + a`` (0-based) holding bit R-1-b of axis a (most significant bit
first).  MPO cores are arrays (w_{l-1}, d_out, d_in, w_l); the operator acts
as (W psi)[s] = sum_t W[s, t] psi[t].

Parity status: ``stencil_mpo`` is pinned by its dense matrix against a
periodic stencil built on the grid directly and by the plane-wave
eigenvalues; ``mpo_apply`` by dense operator times dense vector;
``cubic_step`` by the dense Euler step at full rank on small grids.
"""

import numpy as np

from .aci import aci


def stencil_mpo(R, ndim, axis, weights):
    """MPO of sum_delta w_delta S^delta along ``axis``, delta in (-1, 0, +1),
    with (S^delta psi)(x) = psi(x + delta h) periodically; ``weights`` =
    (w_-1, w_0, w_+1).

    The shift is a binary adder run from the least significant bit (the
    right end of the chain) to the most significant one: the bond carries
    the carry c in {-1, 0, +1}.  At a bit of ``axis`` with output bit s and
    incoming carry c (from the less significant side) the input bit is
    t = (s + c) mod 2 and the outgoing carry floor((s + c) / 2).  Bits of
    other axes pass the carry on unchanged and copy their bit.  The carry
    entering at the least significant bit is delta (weighted by w_delta);
    the carry leaving the most significant bit is dropped (periodicity)."""
    if not 0 <= axis < ndim:
        raise ValueError("axis out of range")
    L = R * ndim
    carries = (-1, 0, 1)
    cores = []
    for site in range(L):
        W = np.zeros((3, 2, 2, 3))          # (carry out, s, t, carry in)
        for ci, c in enumerate(carries):
            for s in range(2):
                if site % ndim == axis:
                    v = s + c
                    t, cout = v % 2, v // 2
                else:
                    t, cout = s, c
                W[carries.index(cout), s, t, ci] = 1.0
        cores.append(W)
    # boundary vectors: drop the final carry on the left, inject delta on the right
    cores[0] = np.einsum("c,cstd->std", np.ones(3), cores[0])[None]
    cores[-1] = np.einsum("cstd,d->cst", cores[-1], np.asarray(weights, dtype=float))[..., None]
    return cores


def laplacian_mpo(R, ndim, axis):
    """Second difference (psi(x+h) - 2 psi(x) + psi(x-h)) / h^2 along axis."""
    inv_h2 = float(4 ** R)
    return stencil_mpo(R, ndim, axis, (inv_h2, -2.0 * inv_h2, inv_h2))


def mpo_apply(W, X):
    """Exact MPO-TT contraction: core l of the result is
    Z[(a, c), s, (b, e)] = sum_t W[a, s, t, b] X[c, t, e], bond index a*r + c
    (the operator's bond major)."""
    out = []
    for Wl, Xl in zip(W, X):
        wa, d, _, wb = Wl.shape
        ra, _, rb = Xl.shape
        Z = np.einsum("astb,cte->acsbe", Wl, Xl)
        out.append(Z.reshape(wa * ra, d, wb * rb))
    return out


def mpo_dense(W):
    """Dense matrix (rows: output index, columns: input index, both in site
    order with the first site most significant) by contracting the chain."""
    M = np.ones((1, 1, 1))                  # (row, col, bond)
    for Wl in W:
        M = np.einsum("rca,astb->rsctb", M, Wl)
        r, s, c, t, b = M.shape
        M = M.reshape(r * s, c * t, b)
    return M[:, :, 0]


def linear_cubic(alpha, beta):
    """f(x^1, ..., x^N) = sum_n alpha_n x^n + beta |x^1|^2 x^1 with
    |z|^2 = re*re + im*im: the right-hand side of an explicit step of a cubic
    equation (the nonlinear term evaluated by ACI, Sec. 4), written as the
    formula reads, the linear terms first and the cubic term last."""
    alpha = list(alpha)

    def f(*P):
        if len(P) != len(alpha):
            raise ValueError("one coefficient per input")
        out = alpha[0] * P[0]
        for c, x in zip(alpha[1:], P[1:]):
            out = out + c * x
        z = P[0]
        a = (z.real * z.real + z.imag * z.imag) if np.iscomplexobj(z) else z * z
        return out + beta * (a * z)

    return f


def cubic_step(psi, R, ndim, c0, c_lap, c3, tol, maxrank, maxiter=20, log_gaps=False):
    """One explicit step y = c0 psi + c_lap sum_a D_a psi + c3 |psi|^2 psi
    (coefficients include the time step), with D_a the periodic second
    difference along axis a.  Returns (ACIResult, [D_a psi])."""
    lap = [mpo_apply(laplacian_mpo(R, ndim, a), psi) for a in range(ndim)]
    f = linear_cubic([c0] + [c_lap] * ndim, c3)
    res = aci([psi] + lap, f, tol, maxrank, maxiter=maxiter, init=psi, log_gaps=log_gaps)
    return res, lap
