"""The oracle's rates at a subset of target particles (used for parity at
sizes the full oracle cannot evolve) are the full rates at those particles,
bit for bit."""
import numpy as np

from paper_2511_22852_amd import inputs as I

from cases import table


def test_rhs_targets_equal_full_rhs(oracle_mod):
    O = oracle_mod
    w = I.lumpy_3d_workload(nxy=16, dxy=0.1, neta=10, deta=0.125, h=0.3, seed=3, n_hot=6, radius=0.6)
    cols, lo, hi = table("small")
    oe = O.eos_table(cols, lo, hi)
    specs = I.jet_sources(seed=12, n_jets=2, radius=0.3, width=0.3, eta_range=0.3, dim=3)
    prm = O.params(dim=3, hyperbolic=True, viscous=True, ncharge=3, h=w.h, use_cells=1, eta_over_s=0.08,
                   zeta_peak=0.02, source_specs=specs)
    y = O.init(prm, oe, w.t0, w.xi, w.u, w.dens_kind, w.dens)
    rng = np.random.default_rng(4)
    for k in range(3):
        y[O.V_U1 + k] += 0.05 * rng.standard_normal(w.n)
    y[O.V_B] = -0.01 * y[O.V_S]
    y[O.V_P12] = 0.02 * y[O.V_S] * rng.standard_normal(w.n)
    f, aux, bad = O.rhs(prm, oe, w.t0, y)
    tg = rng.choice(w.n, 200, replace=False)
    ft, auxt, badt = O.rhs_targets(prm, oe, w.t0, y, tg)
    assert bad == 0 and badt == 0
    assert np.array_equal(ft, f[:, tg])
    assert np.array_equal(auxt, aux[:, tg])
