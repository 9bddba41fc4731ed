"""The allocation-free EoS inversion (ccake_eos_invert_noalloc) against the
ordinary one (ccake_eos_invert) through the C ABI: identical results on two
calls in a row, the second with fewer points (the shared device scratch
keeps the first call's count and must be cleared), and the same error with
the same failure count when inversions are forced to fail from the host
(an iteration limit of one)."""
import numpy as np
import pytest

from paper_2511_22852_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2511_22852_amd import binding
    binding.lib()
    return binding


def points(O, n, seed):
    """(s, nB, nS, nQ) and (e, nB, nS, nQ) of the massless gas (the oracle's
    closed form) at seeded (T, mu), inside and outside the table's range."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(0.06, 0.7, n) / I.HBARC
    mu = rng.uniform(-0.5, 0.5, (3, n)) / I.HBARC
    th = O.eos_eval(O.eos_gas(), False, np.vstack([T, mu]))
    return {0: np.stack([th[2], th[3], th[4], th[5]]), 1: np.stack([th[1], th[3], th[4], th[5]])}


@pytest.mark.parametrize("kind", ["table", "gas"])
def test_noalloc_matches_invert(B, oracle_mod, kind):
    if kind == "table":
        cols, lo, hi = I.massless_gas_table(nT=24, nmu=12)
        eos = B.Eos.table(cols, lo, hi)
    else:
        eos = B.Eos.gas()
    for n, seed in ((6000, 1), (1500, 2)):
        x = points(oracle_mod, n, seed)
        for mode in (0, 1):
            ref, it_ref = eos.invert(mode, 3, x[mode])
            got, it_got = eos.invert(mode, 3, x[mode], noalloc=True)
            assert np.array_equal(got, ref) and np.array_equal(it_got, it_ref), (n, mode)
    eos.close()


def test_noalloc_reports_failures_like_invert(B, oracle_mod):
    eos = B.Eos.gas(max_iter=1, tol=1e-15)
    msgs = []
    for n, seed in ((4000, 3), (700, 4)):
        x = points(oracle_mod, n, seed)
        for noalloc in (False, True):
            with pytest.raises(B.CcakeError) as e:
                eos.invert(0, 3, x[0], noalloc=noalloc)
            assert e.value.status == B.E_EOS_NOCONV
            msgs.append(str(e.value))
    assert msgs[0] == msgs[1] and msgs[2] == msgs[3] and msgs[0] != msgs[2]
    eos.close()
