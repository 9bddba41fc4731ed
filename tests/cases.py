"""Matched parameter sets for the oracle and the HIP library, built from one
description so both sides see identical inputs (test helper)."""
import numpy as np

from paper_2511_22852_amd import inputs as I

TRANSPORT = dict(eta_over_s=0.08, zeta_peak=0.02, zeta_Tpeak_GeV=0.17, zeta_width_GeV=0.02,
                 taupi_coeff=5.0, tauPi_ratio=1.0)
_TABLES = {}


def table(size="small"):
    if size not in _TABLES:
        if size == "small":
            _TABLES[size] = I.massless_gas_table(nT=24, nmu=12)
        else:
            _TABLES[size] = I.massless_gas_table()
    return _TABLES[size]


def make(O, B, *, dim=2, hyperbolic=True, viscous=False, ncharge=0, h=0.3, eos="conformal",
         density_mode=0, precision=0, table_size="small", coeffs=None, skin=None, sources=None,
         diffusion=None):
    """diffusion: None (off) or a dict of kappa_T2, tauJ_coeff, c_JJ (empty
    dict: the defaults of both sides)."""
    tr = dict(TRANSPORT) if viscous else {}
    if coeffs:
        tr.update(coeffs)
    if diffusion is not None:
        tr.update(dict(diffusion=True, **diffusion))
    prm = O.params(dim=dim, hyperbolic=hyperbolic, viscous=viscous, ncharge=ncharge, h=h, use_cells=1,
                   density_mode=density_mode, source_specs=sources, **tr)
    cfg = B.config(dim=dim, hyperbolic=hyperbolic, viscous=viscous, precision=precision, ncharge=ncharge,
                   density_mode=density_mode, h=h, skin=skin, **tr)
    if eos == "conformal":
        oe, ge = O.eos_conformal(11.0), B.Eos.conformal(11.0)
    elif eos == "gas":
        oe, ge = O.eos_gas(), B.Eos.gas()
    else:
        cols, lo, hi = table(table_size)
        oe, ge = O.eos_table(cols, lo, hi), B.Eos.table(cols, lo, hi)
    return prm, oe, cfg, ge


def perturb(O, y, dim, viscous, seed, du=0.05, dpi=0.05):
    """Adds seeded flow and (when viscous) bulk / shear state so that every
    term of the equations of motion is exercised."""
    rng = np.random.default_rng(seed)
    y = y.copy()
    n = y.shape[1]
    for k in range(dim):
        y[O.V_U1 + k] += du * rng.standard_normal(n)
    if viscous:
        S = y[O.V_S]
        y[O.V_B] = -0.3 * dpi * S * rng.random(n)
        rows = [O.V_P11, O.V_P12, O.V_P22, O.V_P33] + ([O.V_P13, O.V_P23] if dim == 3 else [])
        for r in rows:
            y[r] = dpi * S * rng.standard_normal(n)
        if dim == 2:
            y[O.V_P33] /= 0.36  # pi^{eta eta} carries 1/tau^2 at tau ~ 0.6
    return y


def rel_inf(a, b):
    scale = np.abs(b).max()
    if scale == 0.0:
        return np.abs(a).max()
    return np.abs(a - b).max() / scale


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)
