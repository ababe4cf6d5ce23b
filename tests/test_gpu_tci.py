"""2-site TCI on the GPU (aci_tci) against the oracle's (oracle/tci.py).

The test functions are sums of products of one-site tables, evaluated with
the same operations in the same order by NumPy and by torch on the device,
so both sides factorise bit-identical two-site tensors: pivots, ranks,
error estimates and index sets must agree exactly, and the cores to
rounding.  A quantics Gaussian (exp differs in the last bits between the two
libraries) is checked against its closed form."""

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import compare_records

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")


def sum_of_products(G):
    """f(x) = sum_t prod_l G[t, l, x_l], accumulated t ascending, l ascending."""
    T, L, _ = G.shape
    Gd = torch.from_numpy(G).cuda()

    def f_np(pts):
        acc = np.zeros(pts.shape[0], dtype=G.dtype)
        for t in range(T):
            prod = G[t, 0, pts[:, 0]]
            for l in range(1, L):
                prod = prod * G[t, l, pts[:, l]]
            acc = acc + prod
        return acc

    def f_dev(idx):
        idx = idx.long()
        acc = torch.zeros(idx.shape[0], dtype=Gd.dtype, device=idx.device)
        for t in range(T):
            prod = Gd[t, 0][idx[:, 0]]
            for l in range(1, L):
                prod = prod * Gd[t, l][idx[:, l]]
            acc = acc + prod
        return acc

    return f_np, f_dev


@pytest.mark.parametrize("L,d,T,cplx", [(10, 2, 5, False), (8, 3, 4, False), (9, 2, 3, True)])
def test_tci_matches_oracle(L, d, T, cplx):
    rng = np.random.default_rng(100 + L * d + T)
    G = rng.uniform(-1.0, 1.0, (T, L, d))
    if cplx:
        G = G + 1j * rng.uniform(-1.0, 1.0, (T, L, d))
    f_np, f_dev = sum_of_products(G)
    piv = [tuple(rng.integers(0, d, L)) for _ in range(2)]
    ref = oracle.tci(f_np, [d] * L, 1e-12, 32, pivots=piv, log_gaps=True)
    cores, info = aci.tci(f_dev, [d] * L, 1e-12, 32, pivots=piv,
                          dtype=torch.complex128 if cplx else torch.float64)
    assert info.ranks[1:-1] == ref.ranks and info.sweeps == ref.sweeps and info.converged == ref.converged
    np.testing.assert_array_equal(np.array(info.eps), ref.eps)
    for l in range(1, L):
        assert info.I[l] == [tuple(int(v) for v in t) for t in ref.I[l]]
        assert info.J[l + 1] == [tuple(int(v) for v in t) for t in ref.J[l + 1]]
    y = W.tt_full([c.cpu().numpy() for c in cores])
    yr = W.tt_full(ref.cores)
    assert np.abs(y - yr).max() <= 1e-12 * np.abs(yr).max()
    full = f_np(np.stack(np.meshgrid(*[np.arange(d)] * L, indexing="ij"), -1).reshape(-1, L)).reshape([d] * L)
    assert np.abs(y - full).max() <= 1e-10 * np.abs(full).max()


def test_tci_quantics_gaussian():
    R = 14
    w = np.array([2.0 ** -(l + 1) for l in range(R)])
    wd = torch.from_numpy(w).cuda()
    f_dev = lambda idx: torch.exp(-((idx.double() @ wd) - 0.5) ** 2 / (2 * 0.03 ** 2))
    # seeded on both sides of the peak at x = 1/2: from one side only the
    # first bond keeps rank 1 and the other half is never evaluated (a
    # property of TCI, the oracle's run does the same)
    piv = [(1,) + (0,) * (R - 1), (0,) + (1,) * (R - 1)]
    cores, info = aci.tci(f_dev, [2] * R, 1e-10, 64, pivots=piv)
    assert info.converged
    ref = oracle.tci(lambda p: np.exp(-((p @ w) - 0.5) ** 2 / (2 * 0.03 ** 2)), [2] * R, 1e-10, 64, pivots=piv)
    assert info.ranks == [1] + ref.ranks + [1]
    grid = np.stack(np.meshgrid(*[np.arange(2)] * R, indexing="ij"), -1).reshape(-1, R)
    exact = np.exp(-((grid @ w) - 0.5) ** 2 / (2 * 0.03 ** 2))
    got = W.tt_full([c.cpu().numpy() for c in cores]).reshape(-1)
    assert np.abs(got - exact).max() <= 1e-8


def test_tci_evaluator_failure_and_bad_pivots():
    def bad(idx):
        raise RuntimeError("evaluator broke")
    with pytest.raises(RuntimeError, match="evaluator broke"):
        aci.tci(bad, [2] * 6, 1e-10, 8)
    with pytest.raises(Exception, match="INVALID"):
        aci.tci(lambda idx: idx.double().sum(1), [2] * 6, 1e-10, 8, pivots=[(0, 1, 2, 0, 0, 0)])
