"""Pins of the oracle's external source term (eq. conservation_source with
the smeared deposition of the dynamical-initialisation section) against
results fixed by the conservation laws alone:

* Bjorken flow with a uniform source of energy and charge: the interior
  particle of a uniform lattice must follow the closed forms of
  d eps/dtau = -(eps + p)/tau + I^tau and dn_q/dtau = -n_q/tau + I_q
  (eq. e_conservation and eq. charge_conservation with theta = 1/tau) for
  the massless gas (p = eps/3): this pins the 1/sqrt(-g) of the deposition,
  the heating term u.I and the -mu_q I_q term of the entropy equation;
* a static Cartesian medium under a uniform source of energy and x-momentum:
  T^00 and T^0x of the interior particle grow linearly at the source rates
  (eq. conservation_source with vanishing gradients), which pins the sign and
  metric factor of the momentum coupling;
* deposited totals: a localised moving source in a lumpy medium adds exactly
  dN_q/dx0 per unit time to the total charge (up to the lattice quadrature
  of the normalised Gaussian), in Cartesian and hyperbolic coordinates, and
  dp^mu/dx0 to the total energy and momentum in Cartesian coordinates (up to
  the O(dt^2) energy error of the integrator).
"""
import math

import numpy as np

from paper_2511_22852_amd import inputs as I

HBARC = I.HBARC
AG = 19 * math.pi ** 2 / 36


def uniform_lattice(side, dx):
    return I.lattice((side, side), dx, -0.5 * dx * (side - 1))


def gauss2(x, y, centre, width):
    """Value of the normalised 2D Gaussian source profile (input definition)."""
    return math.exp(-((x - centre[0]) ** 2) / (2 * width[0] ** 2) - ((y - centre[1]) ** 2) / (2 * width[1] ** 2)) / (
        2 * math.pi * width[0] * width[1])


def test_bjorken_with_energy_and_charge_source(oracle_mod):
    O = oracle_mod
    T0 = 0.3 / HBARC
    s0 = 4 * AG * T0 ** 3
    side, dx, h = 31, 0.1, 0.15
    xi = uniform_lattice(side, dx)
    n = xi.shape[1]
    dens = np.stack([np.full(n, s0), np.full(n, 0.05 * s0), np.zeros(n), np.full(n, 0.02 * s0)])
    c = int(np.argmin(np.hypot(xi[0], xi[1])))
    width = [1e4, 1e4, 1.0]
    G = gauss2(xi[0, c], xi[1, c], [0.0, 0.0], width)
    A_E, A_B, A_Q = 20.0, 1.0, -0.3          # I^tau = A_E / tau etc. at the particle
    spec = dict(x0=[0, 0, 0], width=width, t_on=0.0, t_off=10.0, dpdt=[A_E / G, 0, 0, 0],
                dndt=[A_B / G, 0.0, A_Q / G])
    prm = O.params(dim=2, hyperbolic=True, viscous=False, ncharge=3, h=h, use_cells=1, source_specs=[spec])
    eos = O.eos_gas()
    t0, dt, nsteps = 1.0, 0.005, 100
    y = O.init(prm, eos, t0, xi, np.zeros_like(xi), 0, dens)
    _, aux0, _ = O.rhs(prm, eos, t0, y)
    t, y, _ = O.evolve(prm, eos, t0, dt, nsteps, y)
    _, aux, _ = O.rhs(prm, eos, t, y)
    e0 = aux0[O.A_E, c]
    r = (t0 / t) ** (4 / 3)
    e_ex = e0 * r + 0.75 * A_E * (1 - r)
    assert abs(aux[O.A_E, c] / e_ex - 1) < 1e-5
    for q, A in ((0, A_B), (2, A_Q)):
        n_ex = (aux0[O.A_NB + q, c] * t0 + A * (t - t0)) / t
        assert abs(aux[O.A_NB + q, c] - n_ex) < 1e-5 * abs(n_ex)
    assert abs(aux[O.A_NS, c]) < 1e-10 * aux[O.A_NB, c]
    # the deposit changed the state well beyond the tolerance
    e_free = e0 * r
    assert abs(e_ex / e_free - 1) > 0.05


def test_static_medium_under_momentum_source(oracle_mod):
    O = oracle_mod
    fstar = 11.0
    side, dx, h = 31, 0.1, 0.15
    xi = uniform_lattice(side, dx)
    n = xi.shape[1]
    e_init = 50.0
    dens = np.stack([np.full(n, e_init), np.zeros(n), np.zeros(n), np.zeros(n)])
    c = int(np.argmin(np.hypot(xi[0], xi[1])))
    width = [1e4, 1e4, 1.0]
    G = gauss2(xi[0, c], xi[1, c], [0.0, 0.0], width)
    I0, Ix = 30.0, 12.0
    spec = dict(x0=[0, 0, 0], width=width, t_on=0.0, t_off=10.0, dpdt=[I0 / G, Ix / G, 0, 0])
    prm = O.params(dim=2, hyperbolic=False, viscous=False, ncharge=0, h=h, use_cells=1, source_specs=[spec])
    eos = O.eos_conformal(fstar)
    t0, dt, nsteps = 0.0, 0.005, 100
    y = O.init(prm, eos, t0, xi, np.zeros_like(xi), 1, dens)
    t, y, _ = O.evolve(prm, eos, t0, dt, nsteps, y)
    _, aux, _ = O.rhs(prm, eos, t, y)
    e, gam, ux = aux[O.A_E, c], aux[O.A_GAMMA, c], y[O.V_U1, c]
    T00 = (4 / 3) * e * gam * gam - e / 3
    T0x = (4 / 3) * e * gam * ux
    assert abs(T00 - (e_init + I0 * (t - t0))) < 1e-6 * T00
    assert abs(T0x - Ix * (t - t0)) < 1e-6 * abs(T0x)
    assert ux > 0.01          # accelerated along +x, as the source pushes
    assert abs(y[O.V_U2, c]) < 1e-12


def lumpy(O, hyperbolic, specs, density_mode, flow=(0.0, 0.0)):
    w = I.lumpy_2d_workload(n_side=40, spacing=0.1, h=0.25, seed=5, n_hot=10, radius=0.8, width=0.5,
                            rhoB=0.02, rhoQ=0.01)
    prm = O.params(dim=2, hyperbolic=hyperbolic, viscous=False, ncharge=3, h=w.h, use_cells=1,
                   density_mode=density_mode, source_specs=specs)
    eos = O.eos_gas()
    t0 = 1.0
    u = np.empty_like(w.xi)
    u[0], u[1] = flow
    y = O.init(prm, eos, t0, w.xi, u, 0, w.dens / 10.0)
    return prm, eos, t0, y


def test_deposited_charge_totals(oracle_mod):
    O = oracle_mod
    dt, nsteps = 0.005, 60
    for hyperbolic in (False, True):
        # charge comes with energy (about 2 GeV per baryon), as stopped baryons do
        spec = dict(x0=[-0.4, 0.1, 0], vel=[0.8, 0.6, 0], width=[0.3, 0.3, 1.0], t_on=1.0525, t_off=1.2525,
                    dpdt=[40.0, 0.0, 0.0, 0.0], dndt=[4.0, 0.0, -1.5])
        # a moving medium (gamma = 1.25): the deposit per particle carries 1/(gamma sigma)
        prm, eos, t0, y = lumpy(O, hyperbolic, [spec], density_mode=1, flow=(0.6, 0.45))
        before = O.totals(prm, eos, t0, y)
        t, y, _ = O.evolve(prm, eos, t0, dt, nsteps, y)
        after = O.totals(prm, eos, t, y)
        dur = 0.2
        assert abs((after[1] - before[1]) - 4.0 * dur) < 2e-3 * 4.0 * dur
        assert abs((after[3] - before[3]) + 1.5 * dur) < 2e-3 * 1.5 * dur
        assert after[2] == before[2]


def test_deposited_energy_momentum_totals(oracle_mod):
    O = oracle_mod
    dt, nsteps = 0.0025, 120
    E, phi = 40.0, 0.7
    spec = dict(x0=[-0.3, 0.0, 0], vel=[math.cos(phi), math.sin(phi), 0], width=[0.3, 0.3, 1.0], t_on=1.00125,
                t_off=1.20125, dpdt=[E, E * math.cos(phi), E * math.sin(phi), 0.0])
    prm, eos, t0, y = lumpy(O, False, [spec], density_mode=1)
    before = O.totals(prm, eos, t0, y)
    t, y, _ = O.evolve(prm, eos, t0, dt, nsteps, y)
    after = O.totals(prm, eos, t, y)
    dep = E * 0.2
    assert abs((after[4] - before[4]) - dep) < 3e-3 * dep
    assert abs((after[5] - before[5]) - dep * math.cos(phi)) < 3e-3 * dep
    assert abs((after[6] - before[6]) - dep * math.sin(phi)) < 3e-3 * dep
    # without the source the same run conserves energy far better than that
    prm0, eos0, _, y0 = lumpy(O, False, [], density_mode=1)
    b0 = O.totals(prm0, eos0, t0, y0)
    _, y1, _ = O.evolve(prm0, eos0, t0, dt, nsteps, y0)
    a0 = O.totals(prm0, eos0, t, y1)
    assert abs(a0[4] - b0[4]) < 3e-4 * dep
