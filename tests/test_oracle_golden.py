"""Pins against numbers the paper prints.

Neighbour estimates (tests/golden/neighbour_estimates.txt, the paper's table
of estimated nearest neighbours): the printed N_nb^est equal the cube
estimate (4h)^3 / (dx_x^2 dx_z), and the oracle's neighbour count (pairs
within the kernel support 2h, self included) at an interior lattice particle
is the ball's share of that cube, pi/6, up to the lattice discretisation.
"""
import math
import os

import numpy as np

from paper_2511_22852_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))


def golden_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "neighbour_estimates.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                n, h, dxx, dxz = line.split()
                rows.append((int(n), float(h), float(dxx), float(dxz)))
    return rows


def test_printed_estimates_are_the_cube_estimate():
    rows = golden_rows()
    assert len(rows) == 3
    for n, h, dxx, dxz in rows:
        assert round((4 * h) ** 3 / (dxx * dxx * dxz)) == n


def test_oracle_neighbour_count_is_the_ball_share(oracle_mod):
    O = oracle_mod
    for n_est, h, dxx, dxz in golden_rows():
        nx = 2 * int(math.ceil(2 * h / dxx)) + 3
        nz = 2 * int(math.ceil(2 * h / dxz)) + 3
        xi = I.lattice((nx, nx, nz), (dxx, dxx, dxz),
                       (-0.5 * dxx * (nx - 1), -0.5 * dxx * (nx - 1), -0.5 * dxz * (nz - 1)))
        c = int(np.argmin((xi ** 2).sum(0)))
        prm = O.params(dim=3, hyperbolic=True, h=h, use_cells=1)
        eos = O.eos_conformal(11.0)
        dens = np.zeros((4, xi.shape[1]))
        dens[0] = 10.0
        y = O.init(prm, eos, 1.0, xi, np.zeros_like(xi), 0, dens)
        _, aux, _ = O.rhs(prm, eos, 1.0, y)
        nnb = aux[O.A_NNB, c]
        # lattice points inside the ball of radius 2h; points on its surface
        # (ties at exactly 2h) fall either way with the rounding of the
        # lattice coordinates
        k = np.arange(-nx, nx + 1)
        kz = np.arange(-nz, nz + 1)
        X, Yy, Z = np.meshgrid(k * dxx, k * dxx, kz * dxz, indexing="ij")
        r2 = X ** 2 + Yy ** 2 + Z ** 2
        inner = int(np.count_nonzero(r2 < (2 * h) ** 2 * (1 - 1e-9)))
        outer = int(np.count_nonzero(r2 < (2 * h) ** 2 * (1 + 1e-9)))
        assert inner <= nnb <= outer, (nnb, inner, outer)
        assert abs(nnb / (math.pi / 6 * n_est) - 1) < 0.05, (nnb, n_est)


def golden_matrix():
    K, tau = [], None
    with open(os.path.join(HERE, "golden", "bsq_diffusion_matrix.txt")) as fh:
        for line in fh:
            if line.startswith("kappa_T2"):
                K.append([float(v) for v in line.split()[1:]])
            elif line.startswith("tau_T"):
                tau = [float(v) for v in line.split()[1:]]
    return np.array(K), np.array(tau)


def test_printed_diffusion_matrix(oracle_mod):
    """The printed kappa/T^2 matrix is the oracle's default, is symmetric
    (Onsager) and positive definite, so the diffusion terms produce entropy:
    -J . grad(alpha) = kappa_{qq'} grad(alpha_q) . grad(alpha_q') >= 0; the
    printed relaxation times are the default tau_J = 0.2 / T."""
    K, tau = golden_matrix()
    assert np.array_equal(np.asarray(oracle_mod.KAPPA_T2_BSQ), K)
    assert np.array_equal(K, K.T)
    assert np.linalg.eigvalsh(K).min() > 0.0
    assert np.all(tau == 0.2)
    prm = oracle_mod.params(dim=2, ncharge=3, diffusion=True)
    assert prm.tauJ_coeff == 0.2 and list(prm.kappa_T2) == list(K.flat)
