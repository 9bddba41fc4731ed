"""GPU parity of the BSQ charge diffusion ("BSQ diffusion", eq. min_dif_rel,
eq. charge_conservation): the HIP library through the C ABI against the
oracle on the same seeded states with random currents J^k_q / sigma.

Bars: rates per state row within 1e-12 normwise (diffusion rows included),
one Heun step within 1e-12, trajectories within 1e-9, charge totals (N_q
plus sqrt(-g) J^0_q / sigma*) within 1e-12, mixed precision within relative
L2 1e-4 of the FP64 oracle on e and n_B; the diffusion sums are FP64 in both precisions.
"""
import numpy as np
import pytest

from cases import make, perturb, rel_inf, rel_l2
from paper_2511_22852_amd import inputs as I

pytestmark = pytest.mark.gpu

DIFF = dict(kappa_T2=4 * np.asarray(((0.0482, -0.0482, 0.0), (-0.0482, 0.1447, 0.0147), (0.0, 0.0147, 0.0880))),
            tauJ_coeff=0.3, c_JJ=0.4)
# with the ADNH coupling of the currents to the bulk-pressure gradient (eq. diffusion-evol)
DIFF_PI = dict(DIFF, d_JPi=(0.2, -0.1, 0.05))


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


def with_currents(O, y, dim, seed, scale=0.01):
    """Seeded random currents J^k_q / sigma of a fraction of each particle's
    own S (currents far above the local entropy drive S negative)."""
    rng = np.random.default_rng(seed)
    y = y.copy()
    S = np.abs(y[O.V_S])
    for q in range(3):
        for k in range(dim):
            y[O.V_JB1 + 3 * q + k] = scale * S * rng.standard_normal(y.shape[1])
    return y


CASES = {
    "2d_milne_viscous_table": dict(dim=2, hyperbolic=True, viscous=True, eos="table"),
    "2d_cartesian_ideal_gas": dict(dim=2, hyperbolic=False, viscous=False, eos="gas"),
    "3d_milne_viscous_table": dict(dim=3, hyperbolic=True, viscous=True, eos="table"),
}


def case_state(O, B, name, precision=0, seed=5, diffusion=DIFF):
    c = CASES[name]
    if c["dim"] == 2:
        w = I.lumpy_2d_workload(n_side=40, seed=seed, n_hot=10, radius=1.0, rhoB=0.005, rhoQ=0.002)
    else:
        w = I.lumpy_3d_workload(nxy=18, dxy=0.1, neta=12, deta=0.125, h=0.3, seed=seed, n_hot=6, radius=0.6,
                                rhoB=0.005, rhoQ=0.002)
    t0 = w.t0 if c["hyperbolic"] else 0.0
    prm, oe, cfg, ge = make(O, B, dim=c["dim"], hyperbolic=c["hyperbolic"], viscous=c["viscous"], ncharge=3,
                            eos=c["eos"], h=w.h, precision=precision, diffusion=diffusion)
    y = O.init(prm, oe, t0, w.xi, w.u, w.dens_kind, w.dens)
    y = perturb(O, y, c["dim"], c["viscous"], seed=seed + 1)
    y = with_currents(O, y, c["dim"], seed=seed + 2)
    return w, t0, prm, oe, cfg, ge, y


@pytest.mark.parametrize("name,diff", [(n, DIFF) for n in CASES] +
                         [(n, DIFF_PI) for n in ("2d_milne_viscous_table", "3d_milne_viscous_table")],
                         ids=list(CASES) + ["2d_milne_viscous_table_dJPi", "3d_milne_viscous_table_dJPi"])
def test_rate_parity(B, O, name, diff):
    w, t0, prm, oe, cfg, ge, y = case_state(O, B, name, diffusion=diff)
    f_o, aux_o, bad = O.rhs(prm, oe, t0, y)
    assert bad == 0
    sim = B.Sim(cfg, ge, w.n)
    sim.set_state(t0, y)
    f_g, aux_g = sim.rhs()
    dim = CASES[name]["dim"]
    for q in range(3):
        for k in range(dim):
            assert np.abs(f_o[O.V_JB1 + 3 * q + k]).max() > 0.0
    for r in range(O.NVAR):
        if np.abs(f_o[r]).max() == 0.0:
            assert np.abs(f_g[r]).max() == 0.0, r
        else:
            assert rel_inf(f_g[r], f_o[r]) <= 1e-12, (r, rel_inf(f_g[r], f_o[r]))
    for a in (O.A_T, O.A_P, O.A_E, O.A_THETA):
        assert rel_inf(aux_g[a], aux_o[a]) <= 1e-12, a
    sim.close()


@pytest.mark.parametrize("diff", [DIFF, DIFF_PI], ids=["kappa", "kappa_dJPi"])
@pytest.mark.parametrize("name", ["2d_milne_viscous_table", "3d_milne_viscous_table"])
def test_heun_step_parity(B, O, name, diff):
    w, t0, prm, oe, cfg, ge, y = case_state(O, B, name, seed=7, diffusion=diff)
    yo, _, bad = O.heun_step(prm, oe, t0, w.dt, y)
    assert bad == 0
    sim = B.Sim(cfg, ge, w.n)
    sim.set_state(t0, y)
    sim.step(w.dt, 1)
    sim.check()
    yg = sim.get_state()
    for r in range(O.NVAR):
        if np.abs(yo[r]).max() > 0.0:
            assert rel_inf(yg[r], yo[r]) <= 1e-12, (r, rel_inf(yg[r], yo[r]))
    sim.close()


@pytest.mark.parametrize("diff", [DIFF, DIFF_PI], ids=["kappa", "kappa_dJPi"])
def test_trajectory_and_totals(B, O, diff):
    w, t0, prm, oe, cfg, ge, y = case_state(O, B, "2d_milne_viscous_table", seed=9, diffusion=diff)
    n = 40
    _, yo, _ = O.evolve(prm, oe, t0, w.dt, n, y)
    sim = B.Sim(cfg, ge, w.n)
    sim.set_state(t0, y)
    sim.step(w.dt, n)
    sim.check()
    yg = sim.get_state()
    for r in (O.V_X1, O.V_U1, O.V_U2, O.V_S, O.V_NB, O.V_NS, O.V_NQ, O.V_B, O.V_P12,
              O.V_JB1, O.V_JB2, O.V_JS1, O.V_JQ2):
        assert rel_inf(yg[r], yo[r]) <= 1e-9, (r, rel_inf(yg[r], yo[r]))
    tot_o = O.totals(prm, oe, t0 + n * w.dt, yo)
    tot_g, _ = sim.totals()
    for k in range(1, 4):
        assert abs(tot_g[k] - tot_o[k]) <= 1e-9 * np.abs(yo[O.V_NB + k - 1]).sum(), k
    sim.close()


@pytest.mark.parametrize("name", ["2d_cartesian_ideal_gas", "3d_milne_viscous_table"])
def test_charge_rates_sum_to_zero(B, O, name):
    """The charge of a particle is N_q + sqrt(-g) J^0_q / sigma* = N_q + Y_q
    with Y_q = (G_k u^k V^k_q) / gamma^2; the n = -1 flux sums move it between
    particles in equal and opposite amounts, so the GPU's rates of N_q + Y_q
    (dY from its own rates of u and V) sum to zero over the event."""
    w, t0, prm, oe, cfg, ge, y = case_state(O, B, name, seed=13)
    dim, hyp = CASES[name]["dim"], CASES[name]["hyperbolic"]
    sim = B.Sim(cfg, ge, w.n)
    sim.set_state(t0, y)
    f, aux = sim.rhs()
    sim.close()
    n = w.n
    G = np.array([1.0, 1.0, t0 * t0 if hyp else 1.0])
    Gd = np.array([0.0, 0.0, 2 * t0 if hyp else 0.0])
    uu, du = np.zeros((3, n)), np.zeros((3, n))
    uu[:dim] = y[O.V_U1:O.V_U1 + dim]
    du[:dim] = f[O.V_U1:O.V_U1 + dim]
    gam = aux[B.AUX_GAMMA]
    dgam = (G[:, None] * uu * du + 0.5 * Gd[:, None] * uu * uu).sum(0) / gam
    for q in range(3):
        V, dV = np.zeros((3, n)), np.zeros((3, n))
        V[:dim] = y[O.V_JB1 + 3 * q:O.V_JB1 + 3 * q + dim]
        dV[:dim] = f[O.V_JB1 + 3 * q:O.V_JB1 + 3 * q + dim]
        X = (G[:, None] * uu * V).sum(0)
        dX = ((Gd[:, None] * uu + G[:, None] * du) * V + G[:, None] * uu * dV).sum(0)
        dY = dX / gam ** 2 - 2 * X * dgam / gam ** 3
        total = (f[O.V_NB + q] + dY).sum()
        assert np.abs(dY).sum() > 1e-3 * np.abs(f[O.V_NB + q]).sum()
        assert abs(total) < 1e-12 * np.abs(f[O.V_NB + q]).sum(), (q, total)


def test_mixed_precision(B, O):
    """Mixed precision (FP32-Kahan pair sums; the diffusion sums stay FP64)
    against the FP64 oracle after 60 steps: relative L2 within 1e-4 on e,
    n_B and the currents."""
    w, t0, prm, oe, cfgm, ge, y = case_state(O, B, "2d_milne_viscous_table", precision=1, seed=11)
    n = 60
    t, yo, _ = O.evolve(prm, oe, t0, w.dt, n, y)
    _, aux_o, bad = O.rhs(prm, oe, t, yo)
    assert bad == 0
    sim = B.Sim(cfgm, ge, w.n)
    sim.set_state(t0, y)
    sim.step(w.dt, n)
    sim.check()
    e_g, nb_g, yg = sim.read(B.AUX_E), sim.read(B.AUX_NB), sim.get_state()
    sim.close()
    assert rel_l2(e_g, aux_o[O.A_E]) <= 1e-4
    assert rel_l2(nb_g, aux_o[O.A_NB]) <= 1e-4
    for r in (O.V_JB1, O.V_JQ2):
        assert rel_l2(yg[r], yo[r]) <= 1e-4, r


def test_diffusion_rejections(B, O):
    ge = B.Eos.gas()
    for bad in (dict(ncharge=0), dict(ncharge=3, tauJ_coeff=0.0), dict(ncharge=3, tauJ_coeff=float("nan"))):
        kw = dict(dim=2, h=0.3, diffusion=True)
        kw.update(bad)
        with pytest.raises(B.CcakeError) as e:
            B.Sim(B.config(**kw), ge, 100)
        assert e.value.status == B.E_ARG
