"""Parity at the full 3+1D sizes: the 1.2 M-particle viscous BSQ event and the
4 M-particle event with jet sources, in the launch configuration the
benchmark times.  The oracle cannot evolve these sizes, so the GPU's own
FP64 state at checkpoints is the common input; the oracle computes the
rates one particle at a time for clustered samples of targets (pass 1 on the
targets and their neighbours), and every rate row of the GPU at those
particles must agree to 1e-12 (normwise over the sample).  The FP32-Kahan
pair sums are checked at the same states: e and n_B within relative L2 1e-4."""
import numpy as np
import pytest

from paper_2511_22852_amd import inputs as I

from cases import make, rel_inf, rel_l2

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


def clustered_targets(xi, n_clusters, per, seed, centres=()):
    """The per nearest particles of each of n_clusters seeded particles and of
    each given centre."""
    rng = np.random.default_rng(seed)
    points = [xi[:, s] for s in rng.choice(xi.shape[1], n_clusters, replace=False)]
    points += [np.asarray(c, dtype=float)[: xi.shape[0]] for c in centres]
    out = []
    for p in points:
        d2 = ((xi - p[:, None]) ** 2).sum(axis=0)
        out.append(np.argpartition(d2, per)[:per])
    return np.unique(np.concatenate(out))


def compare_at(B, O, prm, oe, cfg_mixed, ge, sim, tg, label):
    t = sim.t
    y = sim.get_state()
    f_g, aux_g = sim.rhs()
    f_o, aux_o, bad = O.rhs_targets(prm, oe, t, y, tg)
    assert bad == 0, label
    for r in range(O.NVAR):
        ref, got = f_o[r], f_g[r, tg]
        if np.abs(ref).max() == 0.0:
            assert np.abs(got).max() == 0.0, (label, r)
        else:
            assert rel_inf(got, ref) <= 1e-12, (label, r, rel_inf(got, ref))
    for a in (O.A_SIGSTAR, O.A_S, O.A_T, O.A_E, O.A_THETA):
        assert rel_inf(aux_g[a, tg], aux_o[a]) <= 1e-12, (label, a)
    assert np.array_equal(aux_g[O.A_NNB, tg], aux_o[O.A_NNB]), label
    mixed = B.Sim(cfg_mixed, ge, y.shape[1])
    mixed.set_sources(getattr(sim, "_specs", []))
    mixed.set_state(t, y)
    _, aux_m = mixed.rhs()
    mixed.close()
    for a in (O.A_E, O.A_NB):
        assert rel_l2(aux_m[a, tg], aux_o[a]) <= 1e-4, (label, a, rel_l2(aux_m[a, tg], aux_o[a]))


def run_case(B, O, w, specs, checkpoints, n_clusters, seed):
    kw = dict(dim=3, viscous=True, ncharge=3, eos="table", table_size="full", h=w.h, sources=specs or None)
    prm, oe, cfg, ge = make(O, B, **kw)
    _, _, cfg_m, _ = make(O, B, precision=1, **kw)
    sim = B.Sim(cfg, ge, w.n)
    sim._specs = specs
    if specs:
        sim.set_sources(specs)
    sim.init_particles(w.t0, w.xi, w.u, w.dens_kind, w.dens)
    # samples around seeded particles and around the sources' centres
    tg = clustered_targets(w.xi, n_clusters, 500, seed, centres=[sp["x0"] for sp in specs])
    done = 0
    for c in checkpoints:
        if c > done:
            sim.step(w.dt, c - done)
            sim.check()
            done = c
        compare_at(B, O, prm, oe, cfg_m, ge, sim, tg, f"step {c}")
    sim.close()


def test_lumpy3d_1p2M_sampled_parity(B, O):
    w = I.lumpy_3d_workload()
    assert w.n == 1_228_800
    run_case(B, O, w, [], checkpoints=(0, 5), n_clusters=20, seed=21)


def test_lumpy3d_4M_jets_sampled_parity(B, O):
    w = I.lumpy_3d_source_workload()
    assert w.n == 4_000_000
    run_case(B, O, w, I.jet_sources(), checkpoints=(3,), n_clusters=10, seed=22)
