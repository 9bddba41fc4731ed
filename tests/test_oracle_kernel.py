"""Pins of the oracle's cubic-spline kernel ("Kernel function" section):
unit normalisation in 2D and 3D by quadrature, the gradient against finite
differences of W, continuity at q = 1 and compact support at q = 2."""
import math

import numpy as np
import pytest
from scipy import integrate


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("h", [0.1, 0.24, 0.3])
def test_normalisation(oracle_mod, dim, h):
    W = lambda r: oracle_mod.kernel_w(dim, h, r)
    shell = (lambda r: 2 * math.pi * r) if dim == 2 else (lambda r: 4 * math.pi * r * r)
    # integrate piecewise so the quadrature sees the two polynomial pieces
    tot = sum(integrate.quad(lambda r: shell(r) * W(r), a, b, epsabs=1e-15, epsrel=1e-13)[0]
              for a, b in [(0, h), (h, 2 * h)])
    assert abs(tot - 1.0) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_matches_finite_difference(oracle_mod, dim):
    h = 0.3
    rng = np.random.default_rng(3)
    for r in rng.uniform(0.01, 2 * h - 1e-3, 200):
        eps = 1e-6
        fd = (oracle_mod.kernel_w(dim, h, r + eps) - oracle_mod.kernel_w(dim, h, r - eps)) / (2 * eps)
        an = oracle_mod.kernel_dw_over_r(dim, h, r) * r
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_support_and_continuity(oracle_mod):
    for dim in (2, 3):
        h = 0.3
        sig = 10 / (7 * math.pi * h * h) if dim == 2 else 1 / (math.pi * h ** 3)
        assert oracle_mod.kernel_w(dim, h, 0.0) == pytest.approx(sig, rel=1e-15)
        assert oracle_mod.kernel_w(dim, h, 2 * h) == 0.0
        assert oracle_mod.kernel_w(dim, h, 2.5 * h) == 0.0
        a = oracle_mod.kernel_w(dim, h, h * (1 - 1e-12))
        b = oracle_mod.kernel_w(dim, h, h * (1 + 1e-12))
        assert abs(a - b) < 1e-9 * sig
        assert oracle_mod.kernel_dw_over_r(dim, h, 0.0) == 0.0
        assert oracle_mod.kernel_dw_over_r(dim, h, 2 * h) == 0.0
