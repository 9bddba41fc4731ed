"""Pins of the oracle's Knudsen and inverse Reynolds numbers ("Particlization",
eq. knudsen-reynolds): Kn_pi = tau_pi sqrt(sigma:sigma), Re^-1_pi =
sqrt(pi:pi) / p, Kn_Pi = tau_Pi theta, Re^-1_Pi = |Pi| / p.

Bjorken flow fixes them in closed form: for a fluid at rest in Milne
coordinates, theta = 1/tau and the only shear components are sigma^xx =
sigma^yy = 1/(3 tau), sigma^{eta eta} = -2/(3 tau^3), so sigma:sigma =
2/(3 tau^2); with pi^{ij} given, pi:pi = pi_xx^2 + pi_yy^2 + 2 pi_xy^2 +
tau^4 (pi^{eta eta})^2 (lowered with g = diag(1, -1, -1, -tau^2)).
"""
import math

import numpy as np

from paper_2511_22852_amd import inputs as I


def test_bjorken_closed_forms(oracle_mod):
    O = oracle_mod
    side, dx, h, tau = 31, 0.1, 0.15, 1.3
    xi = I.lattice((side, side), dx, -0.5 * dx * (side - 1))
    n = xi.shape[1]
    c = int(np.argmin(np.hypot(xi[0], xi[1])))
    eta_s, coeff, ratio = 0.2, 5.0, 0.7
    prm = O.params(dim=2, hyperbolic=True, viscous=True, ncharge=0, h=h, eta_over_s=eta_s, taupi_coeff=coeff,
                   tauPi_ratio=ratio, use_cells=1)
    eos = O.eos_conformal(11.0)
    dens = np.stack([np.full(n, 30.0), np.zeros(n), np.zeros(n), np.zeros(n)])
    y = O.init(prm, eos, tau, xi, np.zeros_like(xi), 0, dens)
    yB, p11, p22, p12, p33 = -0.02, 0.05, 0.03, -0.01, -0.04
    y[O.V_B], y[O.V_P11], y[O.V_P22], y[O.V_P12], y[O.V_P33] = yB, p11, p22, p12, p33
    _, aux, bad = O.rhs(prm, eos, tau, y)
    assert bad == 0
    a = lambda r: aux[r, c]
    assert abs(a(O.A_THETA) * tau - 1) < 1e-13
    sig = a(O.A_SIGSTAR) / tau                 # sigma = sigma* / (gamma sqrt(-g)), gamma = 1
    p, e, s = a(O.A_P), a(O.A_E), a(O.A_S)
    taupi = coeff * eta_s * s / (e + p)
    tauPi = ratio * taupi
    assert abs(a(O.A_KN_SHEAR) / (taupi * math.sqrt(2 / 3) / tau) - 1) < 1e-12
    assert abs(a(O.A_KN_BULK) / (tauPi / tau) - 1) < 1e-12
    pipi = sig ** 2 * (p11 ** 2 + p22 ** 2 + 2 * p12 ** 2 + tau ** 4 * p33 ** 2)
    assert abs(a(O.A_REINV_SHEAR) / (math.sqrt(pipi) / p) - 1) < 1e-12
    assert abs(a(O.A_REINV_BULK) / (abs(sig * yB) / p) - 1) < 1e-12


def test_zero_for_ideal_runs(oracle_mod):
    O = oracle_mod
    w = I.lumpy_2d_workload(n_side=16, spacing=0.1, h=0.25, seed=5, n_hot=4, radius=0.8, width=0.5)
    prm = O.params(dim=2, hyperbolic=True, viscous=False, ncharge=0, h=w.h, use_cells=1)
    eos = O.eos_conformal(11.0)
    y = O.init(prm, eos, w.t0, w.xi, w.u, 0, w.dens)
    _, aux, _ = O.rhs(prm, eos, w.t0, y)
    for r in (O.A_KN_SHEAR, O.A_REINV_SHEAR, O.A_KN_BULK, O.A_REINV_BULK):
        assert np.all(aux[r] == 0.0)
