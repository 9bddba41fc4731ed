"""GPU trajectories against the FP64 oracle over many steps, through the
C ABI, in the configurations whose end state the precision gates are quoted
on:

* the ideal shifted-Gubser state in 3+1D ("Code validation", eqs.
  tau_prime, eta_prime, shifted_viscous_Gubser_e/_ur/_utau/_ueta): flow in
  all three directions, binning every few steps with the neighbour rows
  kept between binnings, FP64 within 1e-9 and mixed precision within
  relative L2 1e-4 of e;
* the 40,000-particle viscous BSQ event evolved from tau = 0.6 to 8 fm/c
  (1,480 Heun steps) in the benchmark's launch configuration: FP64 state
  rows within 1e-9 normwise and mixed precision within relative L2 1e-4 on
  e and n_B at the final time.
"""
import numpy as np
import pytest

from cases import make, rel_inf, rel_l2
from paper_2511_22852_amd import inputs as I

pytestmark = pytest.mark.gpu

BENCH_SKIN_H = 0.25   # the benchmark's binning skin of the 2+1D event, in units of h


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


# ------------------------------------------------------- shifted Gubser ----
@pytest.fixture(scope="module")
def shifted_gubser(O):
    """Oracle trajectory of the shifted-Gubser state, tau 1 -> 1.4 fm."""
    w = I.shifted_gubser_workload()
    prm = O.params(dim=3, hyperbolic=True, viscous=False, ncharge=0, h=w.h, use_cells=1)
    oe = O.eos_conformal(11.0)
    y0 = O.init(prm, oe, w.t0, w.xi, w.u, w.dens_kind, w.dens)
    t, yo, _ = O.evolve(prm, oe, w.t0, w.dt, w.nsteps, y0)
    _, aux_o, _ = O.rhs(prm, oe, t, yo)
    return w, y0, t, yo, aux_o


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_shifted_gubser_trajectory(B, O, shifted_gubser, precision):
    """40 steps at dt = 0.01 with skin 0.25 h: the event is binned every
    third step and the neighbour rows of a binning serve the passes of the
    steps after it, so the 3+1D row cache is compared across steps."""
    w, y0, t, yo, aux_o = shifted_gubser
    cfg = B.config(dim=3, hyperbolic=True, viscous=False, ncharge=0, h=w.h, precision=precision,
                   skin=0.25 * w.h)
    sim = B.Sim(cfg, B.Eos.conformal(11.0), w.n)
    sim.set_state(w.t0, y0)
    sim.step(w.dt, w.nsteps)
    sim.check()
    assert abs(sim.t - t) < 1e-12
    yg = sim.get_state()
    e_g = sim.read(B.AUX_E)
    print(f"\nshifted Gubser ({'mixed' if precision else 'fp64'}), {w.n} particles, {w.nsteps} steps:",
          " ".join(f"{r}:{rel_inf(yg[r], yo[r]):.2e}" for r in (O.V_X1, O.V_X3, O.V_U1, O.V_U3, O.V_S)),
          f"e L2 {rel_l2(e_g, aux_o[O.A_E]):.2e}")
    if precision == 0:
        for r in (O.V_X1, O.V_X2, O.V_X3, O.V_U1, O.V_U2, O.V_U3, O.V_S):
            assert rel_inf(yg[r], yo[r]) <= 1e-9, (r, rel_inf(yg[r], yo[r]))
        assert rel_inf(e_g, aux_o[O.A_E]) <= 1e-9
    else:
        assert rel_l2(e_g, aux_o[O.A_E]) <= 1e-4
        for r in (O.V_U1, O.V_U3):
            assert rel_l2(yg[r], yo[r]) <= 1e-4, r


# ------------------------------------------- the 40k event to tau = 8 fm ----
@pytest.fixture(scope="module")
def lumpy_final(O, B):
    """Oracle run of the 40,000-particle event over its full time range
    (tau 0.6 -> 8 fm/c, 1,480 steps; about a minute on 16 host cores)."""
    w = I.lumpy_2d_workload()
    prm, oe, _, _ = make(O, B, dim=2, viscous=True, ncharge=3, eos="table", table_size="full", h=w.h)
    y0 = O.init(prm, oe, w.t0, w.xi, w.u, w.dens_kind, w.dens)
    t, yo, _ = O.evolve(prm, oe, w.t0, w.dt, w.nsteps, y0)
    _, aux_o, bad = O.rhs(prm, oe, t, yo)
    assert bad == 0
    return w, t, yo, aux_o


def run_lumpy(B, O, w, precision):
    _, _, cfg, ge = make(O, B, dim=2, viscous=True, ncharge=3, eos="table", table_size="full", h=w.h,
                         skin=BENCH_SKIN_H * w.h, precision=precision)
    sim = B.Sim(cfg, ge, w.n)
    sim.init_particles(w.t0, w.xi, w.u, w.dens_kind, w.dens)
    sim.step(w.dt, w.nsteps)
    sim.check()
    yg = sim.get_state()
    f, aux_g = sim.rhs()
    t = sim.t
    sim.close()
    return t, yg, aux_g


def test_lumpy_40k_final_time_fp64(B, O, lumpy_final):
    w, t, yo, aux_o = lumpy_final
    tg, yg, aux_g = run_lumpy(B, O, w, B.FP64)
    assert abs(tg - t) < 1e-9 and abs(t - 8.0) < 1e-9
    rows = (O.V_X1, O.V_X2, O.V_U1, O.V_U2, O.V_S, O.V_NB, O.V_NQ, O.V_B, O.V_P11, O.V_P12, O.V_P22, O.V_P33)
    errs = {r: rel_inf(yg[r], yo[r]) for r in rows}
    print("\n40k event at tau = 8 fm (fp64), normwise relative error per row:",
          " ".join(f"{r}:{v:.2e}" for r, v in errs.items()),
          f"e:{rel_inf(aux_g[O.A_E], aux_o[O.A_E]):.2e} T:{rel_inf(aux_g[O.A_T], aux_o[O.A_T]):.2e}")
    for r, v in errs.items():
        assert v <= 1e-9, (r, v)
    for a in (O.A_E, O.A_T, O.A_NB):
        assert rel_inf(aux_g[a], aux_o[a]) <= 1e-9, a


def test_lumpy_40k_final_time_mixed(B, O, lumpy_final):
    w, t, yo, aux_o = lumpy_final
    tg, yg, aux_g = run_lumpy(B, O, w, B.MIXED)
    le, lb = rel_l2(aux_g[O.A_E], aux_o[O.A_E]), rel_l2(aux_g[O.A_NB], aux_o[O.A_NB])
    print(f"\n40k event at tau = 8 fm (mixed): relative L2 e {le:.2e}, n_B {lb:.2e}")
    assert le <= 1e-4 and lb <= 1e-4
    # without diffusion the charges N_q = n_q / sigma ride with the particles:
    # they keep their initial values (set by the FP64 initialisation)
    for r in (O.V_NB, O.V_NS, O.V_NQ):
        assert rel_inf(yg[r], yo[r]) <= 1e-12, r
