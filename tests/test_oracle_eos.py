"""Pins of the oracle's equation of state and inverter ("EoS inverter",
Appendix on the modified conformal EoS).

* table interpolation reproduces the node values of the synthetic massless
  gas exactly, and the oracle's analytic gas matches the independent numpy
  generator of that table;
* Newton on the analytic gas and on the table interpolant recovers (T, mu)
  from (s, n) and (e, n); at mu = 0 it equals the closed form
  T = (s / (4 a_g))^(1/3), a_g = 19 pi^2 / 36;
* the table root agrees with the exact gas root within the interpolation
  error; points whose root lies outside the table axes fall back to the
  analytic gas (backup chain);
* modified conformal EoS: e-mode inversion equals the Appendix's reduction to
  a 1D root in T with the closed-form cubic solution chi_q(T), and the
  minimum energy density eps_min(n) is the T -> 0 limit.
"""
import math

import numpy as np
import pytest
from scipy import optimize

from paper_2511_22852_amd import inputs as I

HBARC = I.HBARC
AG = 19 * math.pi ** 2 / 36


@pytest.fixture(scope="module")
def small_table(oracle_mod):
    cols, lo, hi = I.massless_gas_table(nT=9, nmu=5, T_GeV=(0.1, 0.5), mu_GeV=(-0.3, 0.3))
    return oracle_mod.eos_table(cols, lo, hi), cols, lo, hi


def test_table_nodes_exact(oracle_mod, small_table):
    eos, cols, lo, hi = small_table
    gas = oracle_mod.eos_gas()
    nT, nm = cols.shape[1], cols.shape[2]
    T = np.linspace(lo[0], hi[0], nT)
    m = np.linspace(lo[1], hi[1], nm)
    g = np.stack(np.meshgrid(T, m, m, m, indexing="ij")).reshape(4, -1)
    tab = oracle_mod.eos_eval(eos, True, g)
    ana = oracle_mod.eos_eval(gas, False, g)
    # node values of the table itself: p = T^4 col0, s = T^3 col1, n = T^3 col2..4
    Tn = g[0]
    assert np.allclose(tab[0], Tn ** 4 * cols[0].ravel(), rtol=1e-13, atol=0)
    assert np.allclose(tab[2], Tn ** 3 * cols[1].ravel(), rtol=1e-13, atol=0)
    for q in range(3):
        assert np.allclose(tab[3 + q], Tn ** 3 * cols[2 + q].ravel(), rtol=1e-13, atol=1e-13)
    # the C gas formula equals the independent numpy generator at the nodes
    for r in (0, 2, 3, 4, 5):
        scale = np.abs(ana[r]).max()
        assert np.abs(tab[r] - ana[r]).max() <= 1e-12 * scale


def test_mu0_closed_form(oracle_mod):
    gas = oracle_mod.eos_gas()
    T = np.linspace(0.05, 0.8, 50) / HBARC
    s = 4 * AG * T ** 3
    x = np.stack([s, 0 * s, 0 * s, 0 * s])
    out, _, bad = oracle_mod.eos_invert(gas, 0, 3, x)
    assert bad == 0
    assert np.allclose(out[0], (s / (4 * AG)) ** (1 / 3), rtol=1e-13, atol=0)
    assert np.abs(out[1:]).max() < 1e-12


def test_conformal_closed_form(oracle_mod):
    eos = oracle_mod.eos_conformal(11.0)
    e = np.geomspace(0.01, 100.0, 40)
    T_e = (e / 11.0) ** 0.25
    s = 4 * 11.0 * T_e ** 3 / 3
    x = np.stack([e, 0 * e, 0 * e, 0 * e])
    out, _, _ = oracle_mod.eos_invert(eos, 1, 0, x)
    assert np.allclose(out[0], T_e, rtol=1e-14)
    out, _, _ = oracle_mod.eos_invert(eos, 0, 0, np.stack([s, 0 * s, 0 * s, 0 * s]))
    assert np.allclose(out[0], T_e, rtol=1e-14)


def random_points(n, seed, T=(0.12, 0.55), mu=0.35):
    rng = np.random.default_rng(seed)
    x = np.empty((4, n))
    x[0] = rng.uniform(*T, n) / HBARC
    x[1:] = rng.uniform(-mu, mu, (3, n)) / HBARC
    return x


@pytest.mark.parametrize("mode", [0, 1])
def test_gas_roundtrip(oracle_mod, mode):
    gas = oracle_mod.eos_gas()
    x = random_points(300, 5, mu=0.9)
    th = oracle_mod.eos_eval(gas, False, x)  # p, e, s, nB, nS, nQ
    inp = np.stack([th[2] if mode == 0 else th[1], th[3], th[4], th[5]])
    out, _, bad = oracle_mod.eos_invert(gas, mode, 3, inp)
    assert bad == 0
    assert np.allclose(out[0], x[0], rtol=1e-11)
    assert np.abs(out[1:] - x[1:]).max() < 1e-10 * x[0].max()


def test_table_roundtrip_and_interp_error(oracle_mod):
    cols, lo, hi = I.massless_gas_table(nT=64, nmu=32)
    eos = oracle_mod.eos_table(cols, lo, hi)
    gas = oracle_mod.eos_gas()
    x = random_points(400, 9, T=(0.1, 0.55), mu=0.3)
    th = oracle_mod.eos_eval(eos, True, x)
    out, it, bad = oracle_mod.eos_invert(eos, 0, 3, np.stack([th[2], th[3], th[4], th[5]]))
    assert bad == 0 and it.all()
    assert np.allclose(out[0], x[0], rtol=1e-10)
    assert np.abs(out[1:] - x[1:]).max() < 1e-9 * x[0].max()
    # exact-gas densities: the table root differs from the exact root by the
    # interpolation error only
    thg = oracle_mod.eos_eval(gas, False, x)
    out2, it2, _ = oracle_mod.eos_invert(eos, 0, 3, np.stack([thg[2], thg[3], thg[4], thg[5]]))
    inside = it2.astype(bool)
    assert inside.mean() > 0.9
    assert np.abs(out2[0][inside] / x[0][inside] - 1).max() < 2e-3
    assert np.abs(out2[1:, inside] - x[1:, inside]).max() < 2e-2 * x[0].max()


def test_out_of_table_uses_gas_backup(oracle_mod):
    cols, lo, hi = I.massless_gas_table(nT=64, nmu=32)
    eos = oracle_mod.eos_table(cols, lo, hi)
    gas = oracle_mod.eos_gas()
    s = np.array([175.0, 50.0, 5.0])
    x = np.stack([s, 0.05 * s, 0 * s, 0.02 * s])
    out, it, bad = oracle_mod.eos_invert(eos, 0, 3, x)
    outg, _, _ = oracle_mod.eos_invert(gas, 0, 3, x)
    assert bad == 0 and not it.any()
    assert np.array_equal(out, outg)
    # muB/T ~ 4.7 for these charge fractions (the massless gas)
    assert np.allclose(out[1] / out[0], 4.71, atol=0.02)


def mc_chi(T, n0, A0, beta, c):
    """Appendix: closed-form real root of chi^3 + c beta^2/2 chi - beta^4 n0/(4 A0 T^3) = 0.
    The cubic is odd in (chi, n0); the closed form is evaluated at |n0| (where
    it has no cancellation) and the sign restored."""
    sgn = 1.0 if n0 >= 0 else -1.0
    a1 = 0.5 * c * beta ** 2
    a2 = beta ** 4 * abs(n0) / (4 * A0 * T ** 3)
    d = math.sqrt(12 * a1 ** 3 + 81 * a2 ** 2) + 9 * a2
    return sgn * (2 ** (1 / 3) * d ** (2 / 3) - 2 * 3 ** (1 / 3) * a1) / (6 ** (2 / 3) * d ** (1 / 3))


def test_modified_conformal_appendix(oracle_mod):
    A0, mu0, cq = 2.0, [1.5, 2.0, 2.5], [0.7, 0.4, 0.9]
    eos = oracle_mod.eos_modconf(A0, mu0, cq)
    rng = np.random.default_rng(21)
    for _ in range(20):
        T = rng.uniform(0.5, 3.0)
        mu = rng.uniform(-1.5, 1.5, 3)
        # densities from the Appendix's closed forms (T0 = 1 fm^-1)
        n0 = [2 * A0 * mu[q] / mu0[q] ** 4 * (2 * mu[q] ** 2 + cq[q] * T ** 2 * mu0[q] ** 2) for q in range(3)]
        p = A0 * (T ** 4 + sum((mu[q] / mu0[q]) ** 4 + cq[q] * T ** 2 * (mu[q] / mu0[q]) ** 2 for q in range(3)))
        e0 = 3 * p

        def energy_condition(Tx):
            chis = [mc_chi(Tx, n0[q], A0, mu0[q], cq[q]) for q in range(3)]
            lhs = 1 + sum(cq[q] * chis[q] ** 2 / mu0[q] ** 2 + chis[q] ** 4 / mu0[q] ** 4 for q in range(3))
            return lhs - e0 / (3 * A0 * Tx ** 4)

        Tstar = optimize.brentq(energy_condition, 1e-3, 10.0, xtol=1e-15, rtol=1e-15)
        chis = [mc_chi(Tstar, n0[q], A0, mu0[q], cq[q]) for q in range(3)]
        assert Tstar == pytest.approx(T, rel=1e-10)
        out, _, bad = oracle_mod.eos_invert(eos, 1, 3, np.array([[e0], [n0[0]], [n0[1]], [n0[2]]]))
        assert bad == 0
        assert out[0, 0] == pytest.approx(Tstar, rel=1e-10)
        for q in range(3):
            assert out[1 + q, 0] == pytest.approx(chis[q] * Tstar, rel=1e-9, abs=1e-12)


def test_modified_conformal_eps_min(oracle_mod):
    A0, mu0, cq = 2.0, [1.5, 2.0, 2.5], [0.7, 0.4, 0.9]
    eos = oracle_mod.eos_modconf(A0, mu0, cq)
    n0 = np.array([0.3, -0.2, 0.1])
    eps_min = 3 * A0 * sum((mu0[q] * abs(n0[q]) / (4 * A0)) ** (4 / 3) for q in range(3))
    Ts = []
    for f in (2.0, 1.1, 1.01, 1.0001):
        out, _, bad = oracle_mod.eos_invert(eos, 1, 3, np.array([[f * eps_min], [n0[0]], [n0[1]], [n0[2]]]))
        assert bad == 0
        Ts.append(out[0, 0])
    assert all(a > b for a, b in zip(Ts, Ts[1:]))
    assert Ts[-1] < 0.05 * Ts[0]
