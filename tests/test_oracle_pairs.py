"""Pins of the oracle's neighbour relation: b is a neighbour of a iff
d^2 < (2h)^2 with d^2 accumulated axis by axis in FP64 (self included).
Checked by an independent numpy brute force on tiny inputs, including a
lattice where many pairs sit exactly at 2h; the oracle's uniform-grid search
must return the identical pair set."""
import numpy as np
import pytest

from paper_2511_22852_amd import inputs as I


def numpy_pairs(x, h):
    n = x.shape[1]
    d2 = np.zeros((n, n))
    for k in range(x.shape[0]):
        dx = x[k][:, None] - x[k][None, :]
        d2 = d2 + dx * dx
    a, b = np.nonzero(d2 < (2.0 * h) * (2.0 * h))
    return set(zip(a.tolist(), b.tolist()))


def state_from(oracle_mod, x):
    y = np.zeros((oracle_mod.NVAR, x.shape[1]))
    y[: x.shape[0]] = x
    return y


@pytest.mark.parametrize("dim,n,box,h", [(2, 600, 4.0, 0.24), (3, 500, 2.0, 0.3), (2, 1, 1.0, 0.3)])
@pytest.mark.parametrize("cells", [0, 1])
def test_random_cloud(oracle_mod, dim, n, box, h, cells):
    x = I.random_cloud(n, dim, box, seed=11 + dim)
    prm = oracle_mod.params(dim=dim, h=h, use_cells=cells)
    a, b = oracle_mod.pairs(prm, state_from(oracle_mod, x))
    got = list(zip(a.tolist(), b.tolist()))
    assert got == sorted(got)
    assert set(got) == numpy_pairs(x, h)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("cells", [0, 1])
def test_exact_2h_ties(oracle_mod, dim, cells):
    # 2h = 3 * spacing: every third lattice neighbour sits at distance 2h
    side = 14 if dim == 2 else 7
    x = I.tie_lattice(side, 0.1, dim, jitter=0.0, seed=0)
    prm = oracle_mod.params(dim=dim, h=0.15, use_cells=cells)
    a, b = oracle_mod.pairs(prm, state_from(oracle_mod, x))
    got = set(zip(a.tolist(), b.tolist()))
    assert got == numpy_pairs(x, 0.15)
    # symmetric relation, self included
    assert all((j, i) in got for (i, j) in got)
    assert all((i, i) in got for i in range(x.shape[1]))


def test_grid_matches_brute_force_on_lumpy_lattice(oracle_mod):
    w = I.lumpy_2d_workload(n_side=60)
    y = state_from(oracle_mod, w.xi)
    pa = oracle_mod.pairs(oracle_mod.params(dim=2, h=w.h, use_cells=0), y)
    pb = oracle_mod.pairs(oracle_mod.params(dim=2, h=w.h, use_cells=1), y)
    assert np.array_equal(pa[0], pb[0]) and np.array_equal(pa[1], pb[1])
