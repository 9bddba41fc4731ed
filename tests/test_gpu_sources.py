"""GPU parity of the external source term (eq. conservation_source with the
smeared deposition): the HIP library against the FP64 oracle with jet and
stopped-baryon sources, for the rates, one Heun step and a trajectory that
crosses the sources' switch-on and switch-off.  Bars as for the other FP64
parity tests: 1e-12 per stage, 1e-9 on trajectories."""
import numpy as np
import pytest

from paper_2511_22852_amd import inputs as I

from cases import make, perturb, rel_inf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2511_22852_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


def lumpy2d():
    return I.lumpy_2d_workload(n_side=48, seed=1, n_hot=10, radius=1.0, rhoB=0.005, rhoQ=0.002)


def lumpy3d():
    return I.lumpy_3d_workload(nxy=20, dxy=0.1, neta=12, deta=0.125, h=0.3, seed=3, n_hot=6, radius=0.6)


def jets2d():
    return I.jet_sources(seed=11, n_jets=4, radius=0.6, width=0.3, dim=2)


def jets3d():
    return I.jet_sources(seed=12, n_jets=4, radius=0.4, width=0.3, eta_range=0.5, dim=3)


def sheets3d():
    return I.baryon_stopping_sources(n_baryons=20.0, eta0=0.4, width_eta=0.3, radius=0.8)


CASES = {
    "lumpy2d_visc_table_jets": dict(wl=lumpy2d, src=jets2d,
                                    kw=dict(dim=2, viscous=True, ncharge=3, eos="table", h=0.24), visc=True),
    "lumpy2d_ideal_gas_cartesian_charged": dict(
        wl=lumpy2d, src=lambda: [dict(x0=[0.2, -0.1, 0], vel=[0.5, 0.5, 0], width=[0.4, 0.3, 1.0], t_on=0.9,
                                      t_off=5.0, dpdt=[30.0, 5.0, -3.0, 0.0], dndt=[2.0, -0.5, 1.0])],
        kw=dict(dim=2, hyperbolic=False, ncharge=3, eos="gas", h=0.24), visc=False),
    "lumpy3d_visc_table_jets_sheets": dict(wl=lumpy3d, src=lambda: jets3d() + sheets3d(),
                                           kw=dict(dim=3, viscous=True, ncharge=3, eos="table", h=0.3),
                                           visc=True),
}


def prepared(B, O, name):
    c = CASES[name]
    w = c["wl"]()
    specs = c["src"]()
    kw = dict(c["kw"])
    prm, oe, cfg, ge = make(O, B, sources=specs, **kw)
    t0 = w.t0 if kw.get("hyperbolic", True) else 1.0
    y = O.init(prm, oe, t0, w.xi, w.u, w.dens_kind, w.dens)
    y = perturb(O, y, kw["dim"], c["visc"], seed=9)
    return prm, oe, cfg, ge, y, t0, specs, w


def sim_with(B, cfg, ge, y, t, specs):
    s = B.Sim(cfg, ge, y.shape[1])
    s.set_state(t, y)
    s.set_sources(specs)
    return s


@pytest.mark.parametrize("name", list(CASES))
def test_rate_parity_with_sources(B, O, name):
    prm, oe, cfg, ge, y, t0, specs, _ = prepared(B, O, name)
    f_o, aux_o, bad = O.rhs(prm, oe, t0, y)
    assert bad == 0
    # the sources act: the rates differ from the source-free ones
    prm0, oe0, _, _ = make(O, B, **CASES[name]["kw"])
    f_0, _, _ = O.rhs(prm0, oe0, t0, y)
    assert rel_inf(f_0[O.V_S], f_o[O.V_S]) > 1e-6
    sim = sim_with(B, cfg, ge, y, t0, specs)
    f_g, aux_g = sim.rhs()
    for r in range(O.NVAR):
        if np.abs(f_o[r]).max() == 0.0:
            assert np.abs(f_g[r]).max() == 0.0, r
        else:
            assert rel_inf(f_g[r], f_o[r]) <= 1e-12, (r, rel_inf(f_g[r], f_o[r]))
    for a in (O.A_SIGSTAR, O.A_S, O.A_T, O.A_P, O.A_E, O.A_THETA):
        assert rel_inf(aux_g[a], aux_o[a]) <= 1e-12, a


@pytest.mark.parametrize("name", list(CASES))
def test_heun_step_with_sources(B, O, name):
    prm, oe, cfg, ge, y, t0, specs, _ = prepared(B, O, name)
    dt = 0.005
    yo, _, bad = O.heun_step(prm, oe, t0, dt, y)
    assert bad == 0
    sim = sim_with(B, cfg, ge, y, t0, specs)
    sim.step(dt, 1)
    sim.check()
    yg = sim.get_state()
    for r in range(O.NVAR):
        if np.abs(yo[r]).max() > 0:
            assert rel_inf(yg[r], yo[r]) <= 1e-12, (r, rel_inf(yg[r], yo[r]))


def test_source_window_trajectory(B, O):
    """30 Heun steps of the 2D viscous BSQ event with two jets that switch on
    and off inside the run (windows centred between steps), then removal of
    the sources: the remaining steps must follow the source-free oracle."""
    w = lumpy2d()
    specs = jets2d()[:2]
    for sp in specs:
        sp["t_on"], sp["t_off"] = w.t0 + 0.0325, w.t0 + 0.1025
    prm, oe, cfg, ge = make(O, B, dim=2, viscous=True, ncharge=3, eos="table", h=w.h, sources=specs)
    y = O.init(prm, oe, w.t0, w.xi, w.u, w.dens_kind, w.dens)
    t, yo, _ = O.evolve(prm, oe, w.t0, w.dt, 30, y)
    sim = B.Sim(cfg, ge, w.n)
    sim.init_particles(w.t0, w.xi, w.u, w.dens_kind, w.dens)
    sim.set_sources(specs)
    sim.step(w.dt, 30)
    sim.check()
    yg = sim.get_state()
    for r in (O.V_X1, O.V_U1, O.V_U2, O.V_S, O.V_NB, O.V_NQ, O.V_B, O.V_P11, O.V_P12):
        assert rel_inf(yg[r], yo[r]) <= 1e-9, (r, rel_inf(yg[r], yo[r]))
    prm0, oe0, _, _ = make(O, B, dim=2, viscous=True, ncharge=3, eos="table", h=w.h)
    _, yo2, _ = O.evolve(prm0, oe0, t, w.dt, 10, yo)
    sim.set_sources([])
    sim.step(w.dt, 10)
    sim.check()
    yg2 = sim.get_state()
    for r in (O.V_X1, O.V_U1, O.V_S, O.V_NB):
        assert rel_inf(yg2[r], yo2[r]) <= 1e-9, (r, rel_inf(yg2[r], yo2[r]))


def test_rejects_bad_sources(B, O):
    prm, oe, cfg, ge, y, t0, specs, _ = prepared(B, O, "lumpy2d_visc_table_jets")
    sim = B.Sim(cfg, ge, y.shape[1])
    sim.set_state(t0, y)
    with pytest.raises(B.CcakeError):
        sim.set_sources([dict(width=[0.0, 0.3, 0.3])])
    with pytest.raises(B.CcakeError):
        sim.set_sources([dict(width=[0.3, 0.3, 0.3])] * (B.MAX_SOURCES + 1))
