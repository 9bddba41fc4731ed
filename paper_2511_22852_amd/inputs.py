"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds input recipes only -- particle lattices, initial profiles,
the synthetic equation-of-state table -- and none of the SPH method's
arithmetic.  Every generator is deterministic in its seed (numpy PCG64).

The paper's own initial-state generators (TRENTo, AMPT) and lattice-QCD EoS
tables are not available; these stand-ins follow the shapes the paper uses:
lattice initial conditions ("Convergence Tests"), Gaussian hot-spot structure,
h = 0.24-0.3 fm, and for the EoS a 4D (T, muB, muS, muQ) table.

Units: hbar = c = 1, lengths in fm, energies in fm^-1 unless a name says GeV.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

HBARC = 0.1973269804  # GeV fm

# ---------------------------------------------------------------------------
# lattices
# ---------------------------------------------------------------------------


def lattice(shape, spacing, origin):
    """Regular lattice with the first axis varying fastest: returns (D, N)
    positions x_k = origin_k + spacing_k * i_k."""
    shape = tuple(int(s) for s in shape)
    D = len(shape)
    spacing = np.broadcast_to(np.asarray(spacing, float), (D,))
    origin = np.broadcast_to(np.asarray(origin, float), (D,))
    idx = np.indices(tuple(reversed(shape))).reshape(D, -1)
    out = np.empty((D, idx.shape[1]))
    for k in range(D):
        out[k] = origin[k] + spacing[k] * idx[D - 1 - k]
    return out


def random_cloud(n, dim, box, seed):
    """n uniform points in [-box/2, box/2)^dim, seed PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-box / 2, box / 2, size=(dim, n))


def tie_lattice(n_side, spacing, dim, jitter, seed):
    """Lattice whose spacing makes many pairs sit exactly at 2h when
    2h is a multiple of the spacing; optional jitter of a few particles."""
    x = lattice((n_side,) * dim, spacing, -0.5 * spacing * (n_side - 1))
    if jitter > 0:
        rng = np.random.Generator(np.random.PCG64(seed))
        idx = rng.choice(x.shape[1], size=max(1, x.shape[1] // 10), replace=False)
        x[:, idx] += rng.uniform(-jitter, jitter, size=(dim, idx.size))
    return x


# ---------------------------------------------------------------------------
# Gubser flow initial condition (ideal, conformal; "Code validation")
# ---------------------------------------------------------------------------


def gubser_ideal(tau, x, y, q=1.0, That0=None, e_ref_GeV=10.0):
    """Ideal Gubser flow: energy density [fm^-4] and (u^x, u^y) at proper time
    tau [fm].  T_G = That(rho) / (f*^(1/4) tau) with That = That0 /
    cosh(rho)^(2/3), sinh(rho) = (q^2 (tau^2 - r^2) - 1) / (2 q tau); the
    energy density f* T_G^4 is independent of f*.  That0 defaults to the value
    that puts e(tau=1 fm, r=0) at e_ref_GeV GeV/fm^3."""
    if That0 is None:
        That0 = (e_ref_GeV / HBARC) ** 0.25
    r2 = x * x + y * y
    r = np.sqrt(r2)
    sinh_rho = (q * q * (tau * tau - r2) - 1.0) / (2.0 * q * tau)
    cosh_rho = np.sqrt(1.0 + sinh_rho * sinh_rho)
    e = That0 ** 4 / (tau ** 4 * cosh_rho ** (8.0 / 3.0))
    den = np.sqrt(1.0 + 2.0 * q * q * (tau * tau + r2) + q ** 4 * (tau * tau - r2) ** 2)
    ur = 2.0 * q * q * r * tau / den
    with np.errstate(invalid="ignore", divide="ignore"):
        ux = np.where(r > 0, ur * x / np.where(r > 0, r, 1.0), 0.0)
        uy = np.where(r > 0, ur * y / np.where(r > 0, r, 1.0), 0.0)
    return e, ux, uy


def shifted_gubser_ideal(tau, x, y, eta, t_shift=0.5, q=1.0, e_ref_GeV=80.0):
    """Ideal Gubser flow translated in Minkowski time, t -> t + t_shift
    ("Code validation", eqs. tau_prime, eta_prime and
    shifted_viscous_Gubser_e, _ur, _utau, _ueta): with
    tau' = sqrt(tau^2 + 2 t_shift tau cosh(eta) + t_shift^2),
        e = e_G(tau', r),  u^r = u^r_G(tau', r),
        u^eta = -u^tau_G(tau', r) t_shift sinh(eta) / (tau tau').
    The Gubser solution is normalised so that e_G(tau' = 1 fm, r = 0) =
    e_ref_GeV GeV/fm^3, i.e. the shifted one has that value at
    (tau, r, eta) = (1 fm - t_shift, 0, 0), the paper's normalisation point
    for t_shift = 0.5 fm.  Returns e [fm^-4] and (u^x, u^y, u^eta)."""
    taup = np.sqrt(tau * tau + 2.0 * t_shift * tau * np.cosh(eta) + t_shift * t_shift)
    e, ux, uy = gubser_ideal(taup, x, y, q=q, e_ref_GeV=e_ref_GeV)
    r2 = x * x + y * y
    den = np.sqrt(1.0 + 2.0 * q * q * (taup * taup + r2) + q ** 4 * (taup * taup - r2) ** 2)
    utau_g = (1.0 + q * q * (taup * taup + r2)) / den
    ueta = -utau_g * t_shift * np.sinh(eta) / (tau * taup)
    return e, ux, uy, ueta


@dataclass
class Workload:
    """A ready-to-run particle set: positions (D, n), flow u^i (D, n),
    densities (4, n) = (s or e, nB, nS, nQ), dens_kind 0 = s, 1 = e."""
    name: str
    dim: int
    hyperbolic: bool
    xi: np.ndarray
    u: np.ndarray
    dens: np.ndarray
    dens_kind: int
    t0: float
    dt: float
    nsteps: int
    h: float
    viscous: bool
    ncharge: int
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.xi.shape[1]


def gubser_workload(n_side=51, spacing=0.2, h=0.3, hyperbolic=True, t0=1.0, dt=0.005, t_end=2.0):
    """51 x 51 lattice of spacing 0.2 fm, Gubser IC at tau0 = 1 fm, q = 1/fm,
    e(1, 0) = 10 GeV/fm^3; conformal EoS f* = 11, ideal, no charges."""
    half = 0.5 * spacing * (n_side - 1)
    xi = lattice((n_side, n_side), spacing, -half)
    e, ux, uy = gubser_ideal(t0, xi[0], xi[1])
    dens = np.zeros((4, xi.shape[1]))
    dens[0] = e
    return Workload("gubser_2d", 2, hyperbolic, xi, np.stack([ux, uy]), dens, 1, t0, dt,
                    int(round((t_end - t0) / dt)), h, False, 0)


def shifted_gubser_workload(spacing=0.2, deta=0.2, h=0.3, half_xy=3.2, half_eta=1.6, t0=1.0, dt=0.01,
                            t_end=1.4, t_shift=0.5):
    """3+1D lattice in (x, y, eta) with the ideal shifted-Gubser state at
    tau0 = 1 fm (t_shift = 0.5 fm, q = 1/fm, e_G(tau' = 1, 0) = 80 GeV/fm^3,
    the paper's "Code validation" set-up on a smaller box and a coarser
    lattice); conformal EoS f* = 11, ideal, no charges."""
    nxy = int(round(2 * half_xy / spacing)) + 1
    neta = int(round(2 * half_eta / deta)) + 1
    xi = lattice((nxy, nxy, neta), (spacing, spacing, deta), (-half_xy, -half_xy, -half_eta))
    e, ux, uy, ueta = shifted_gubser_ideal(t0, xi[0], xi[1], xi[2], t_shift=t_shift)
    dens = np.zeros((4, xi.shape[1]))
    dens[0] = e
    return Workload("shifted_gubser_3d", 3, True, xi, np.stack([ux, uy, ueta]), dens, 1, t0, dt,
                    int(round((t_end - t0) / dt)), h, False, 0, extra=dict(t_shift=t_shift))


# ---------------------------------------------------------------------------
# Lumpy (hot-spot) initial conditions
# ---------------------------------------------------------------------------


def hotspot_field(x, y, centers, width):
    """H(x) = sum_k exp(-|x - c_k|^2 / (2 width^2)), evaluated in chunks."""
    H = np.zeros(x.shape[0])
    for c in centers:
        H += np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2) / (2.0 * width * width))
    return H


def lumpy_profile(xi, n_hot, radius, width, seed, s0=175.0, floor=0.01):
    rng = np.random.Generator(np.random.PCG64(seed))
    centers = rng.normal(0.0, radius, size=(n_hot, 2))
    H = hotspot_field(xi[0], xi[1], centers, width)
    return floor * s0 + s0 * H / H.max(), centers


def lumpy_2d_workload(n_side=200, spacing=0.08, h=0.24, seed=1, n_hot=150, radius=3.0,
                      width=0.5, rhoB=0.05, rhoQ=0.02, t0=0.6, dt=0.005, t_end=8.0,
                      name="lumpy_2d"):
    """2+1D boost-invariant viscous BSQ event on a square lattice of spacing
    0.08 fm (200 x 200 = 40,000 particles on [-8, 8)^2): s = 0.01 s0 +
    s0 H / max H with s0 = 175 fm^-3 (T ~ 0.4 GeV at mu = 0), 150 hot spots
    of width 0.5 fm centred ~ N(0, 3^2); rhoB = 0.05 s, rhoS = 0,
    rhoQ = 0.02 s; u = 0."""
    half = 0.5 * spacing * n_side
    xi = lattice((n_side, n_side), spacing, -half)
    s, _ = lumpy_profile(xi, n_hot, radius, width, seed)
    dens = np.stack([s, rhoB * s, np.zeros_like(s), rhoQ * s])
    return Workload(name, 2, True, xi, np.zeros_like(xi), dens, 0, t0, dt,
                    int(round((t_end - t0) / dt)), h, True, 3,
                    {"seed": seed, "n_hot": n_hot, "radius": radius})


def serving_events(n_events=256, seed_base=1000, arrival_seed=7, nmin=5000, nmax=80000):
    """Event sizes N_k ~ U{5000..80000} (seed PCG64(seed_base + k)), each a
    square lattice with round(sqrt(N_k)) particles per side at 0.08 fm,
    150 N_k / 40000 hot spots within radius 3 sqrt(N_k / 40000) fm."""
    specs = []
    for k in range(n_events):
        rng = np.random.Generator(np.random.PCG64(seed_base + k))
        N = int(rng.integers(nmin, nmax + 1))
        side = int(round(np.sqrt(N)))
        scale = side * side / 40000.0
        specs.append(dict(k=k, n_side=side, seed=seed_base + k,
                          n_hot=max(1, int(round(150 * scale))),
                          radius=3.0 * np.sqrt(scale)))
    return specs


def serving_event(spec, rhoB=0.05, rhoQ=0.02):
    return lumpy_2d_workload(n_side=spec["n_side"], seed=spec["seed"], n_hot=spec["n_hot"],
                             radius=spec["radius"], rhoB=rhoB, rhoQ=rhoQ,
                             name=f"event_{spec['k']}")


def poisson_arrivals(n, rate, seed=7):
    """Arrival times (s) of a Poisson process with the given rate (1/s)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def lumpy_3d_workload(nxy=160, dxy=0.1, neta=48, deta=0.125, h=0.3, seed=2, n_hot=150,
                      radius=3.0, width=0.5, rhoB=0.05, rhoQ=0.02, t0=0.6, dt=0.005,
                      plateau=1.5, tail=0.5, name="lumpy_3d"):
    """3+1D hyperbolic (tau, x, y, eta) event: the 2D lumpy profile on
    [-8, 8)^2 at 0.1 fm times a plateau-Gaussian in eta (flat for |eta| <
    1.5, Gaussian tails of width 0.5), eta on [-3, 3) at 0.125."""
    xi2 = lattice((nxy, nxy), dxy, -0.5 * dxy * nxy)
    s2, _ = lumpy_profile(xi2, n_hot, radius, width, seed)
    etas = -0.5 * deta * neta + deta * np.arange(neta)
    prof = np.where(np.abs(etas) < plateau, 1.0, np.exp(-(np.abs(etas) - plateau) ** 2 / (2 * tail * tail)))
    n2 = xi2.shape[1]
    xi = np.empty((3, n2 * neta))
    xi[0] = np.tile(xi2[0], neta)
    xi[1] = np.tile(xi2[1], neta)
    xi[2] = np.repeat(etas, n2)
    s = np.tile(s2, neta) * np.repeat(prof, n2)
    dens = np.stack([s, rhoB * s, np.zeros_like(s), rhoQ * s])
    return Workload(name, 3, True, xi, np.zeros_like(xi), dens, 0, t0, dt, 0, h, True, 3,
                    {"seed": seed})


def jet_sources(seed=4, n_jets=4, E_GeV=20.0, t_on=0.6, duration=2.0, width=0.3, radius=3.0,
                eta_range=1.0, dim=3):
    """External energy-momentum sources for jets: n_jets/2 back-to-back pairs
    from seeded production points (transverse ~ N(0, radius^2) per axis, eta
    ~ U(-eta_range, eta_range) in 3D), directions phi ~ U(0, 2 pi) and phi + pi,
    moving transversely at the speed of light.  Each deposits E_GeV uniformly
    over [t_on, t_on + duration) through a Gaussian of the given width, with
    the momentum of a massless particle at its own rapidity (p^eta = 0).
    Returns source dicts (x0, vel, width, t_on, t_off, dpdt, dndt)."""
    rng = np.random.default_rng(seed)
    rate = E_GeV / HBARC / duration
    specs = []
    for _ in range(n_jets // 2):
        x, y = rng.normal(0.0, radius, 2)
        eta = rng.uniform(-eta_range, eta_range) if dim == 3 else 0.0
        phi = rng.uniform(0.0, 2.0 * np.pi)
        for ph in (phi, phi + np.pi):
            c, sn = float(np.cos(ph)), float(np.sin(ph))
            specs.append(dict(x0=[float(x), float(y), float(eta)], vel=[c, sn, 0.0], width=[width] * 3,
                              t_on=t_on, t_off=t_on + duration, dpdt=[rate, rate * c, rate * sn, 0.0],
                              dndt=[0.0, 0.0, 0.0]))
    return specs


def baryon_stopping_sources(n_baryons=100.0, eta0=1.0, width_eta=0.3, radius=3.0, t_on=0.6, duration=2.0,
                            E_per_baryon_GeV=0.94):
    """Stopped-baryon variant: baryon number deposited at rest on the sheets
    eta_s = +-eta0 (Gaussian in eta of width width_eta, transverse Gaussian of
    width radius), n_baryons in total over [t_on, t_on + duration), each with
    the nucleon rest energy.  Returns source dicts."""
    rate_B = 0.5 * n_baryons / duration
    rate_E = rate_B * E_per_baryon_GeV / HBARC
    return [dict(x0=[0.0, 0.0, sgn * eta0], vel=[0.0, 0.0, 0.0], width=[radius, radius, width_eta], t_on=t_on,
                 t_off=t_on + duration, dpdt=[rate_E, 0.0, 0.0, 0.0], dndt=[rate_B, 0.0, 0.0])
            for sgn in (1.0, -1.0)]


def lumpy_3d_source_workload(nxy=200, dxy=0.1, neta=100, deta=0.06, h=0.3, seed=4, **kw):
    """The 4.0 M-particle 3+1D event of the jet-source runs: the lumpy profile
    on [-10, 10)^2 at 0.1 fm times the eta plateau, eta on [-3, 3) at 0.06."""
    return lumpy_3d_workload(nxy=nxy, dxy=dxy, neta=neta, deta=deta, h=h, seed=seed,
                             name="lumpy_3d_sources", **kw)


# ---------------------------------------------------------------------------
# Synthetic 4D EoS table: massless u, d, s quarks + gluons
# ---------------------------------------------------------------------------

FLAVOURS = np.array([[1 / 3, 0.0, 2 / 3], [1 / 3, 0.0, -1 / 3], [1 / 3, -1.0, -1 / 3]])


def massless_gas_table(nT=64, nmu=32, T_GeV=(0.05, 0.6), mu_GeV=(-0.4, 0.4)):
    """Columns (7, nT, nmu, nmu, nmu) of the massless 3-flavour + gluon gas on
    a regular (T, muB, muS, muQ) grid: p/T^4, s/T^3, nB/T^3, nS/T^3, nQ/T^3,
    c_s^2 (= 1/3), (dp/de)_n (= 1/3).  Returns (cols, lo_fm, hi_fm)."""
    lo = np.array([T_GeV[0], mu_GeV[0], mu_GeV[0], mu_GeV[0]]) / HBARC
    hi = np.array([T_GeV[1], mu_GeV[1], mu_GeV[1], mu_GeV[1]]) / HBARC
    T = np.linspace(lo[0], hi[0], nT)[:, None, None, None]
    mB = np.linspace(lo[1], hi[1], nmu)[None, :, None, None]
    mS = np.linspace(lo[2], hi[2], nmu)[None, None, :, None]
    mQ = np.linspace(lo[3], hi[3], nmu)[None, None, None, :]
    ag = 19.0 * np.pi ** 2 / 36.0
    shape = (nT, nmu, nmu, nmu)
    p = np.broadcast_to(ag * T ** 4, shape).copy()
    s = np.broadcast_to(4.0 * ag * T ** 3, shape).copy()
    n = np.zeros((3,) + shape)
    for f in range(3):
        mf = FLAVOURS[f, 0] * mB + FLAVOURS[f, 1] * mS + FLAVOURS[f, 2] * mQ
        p += 0.5 * mf ** 2 * T ** 2 + mf ** 4 / (4.0 * np.pi ** 2)
        s += mf ** 2 * T
        nf = mf * T ** 2 + mf ** 3 / np.pi ** 2
        for q in range(3):
            n[q] += FLAVOURS[f, q] * nf
    cols = np.empty((7,) + shape)
    cols[0] = p / T ** 4
    cols[1] = s / T ** 3
    for q in range(3):
        cols[2 + q] = n[q] / T ** 3
    cols[5] = 1.0 / 3.0
    cols[6] = 1.0 / 3.0
    return cols, lo, hi
