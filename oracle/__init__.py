"""Plain FP64 CPU oracle for the CCAKE 2.0 SPH stage (arXiv 2511.22852).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only permitted callers.  The
product path (``paper_2511_22852_amd``) never imports this package and shares
no code with it.

The arithmetic lives in ``ccake_oracle.c`` (compiled with gcc, no FMA
contraction, OpenMP over particles); this module only marshals numpy arrays.
Units: hbar = c = 1, fm.  Table axes and zeta/s parameters are accepted in GeV
and converted with hbar*c = 0.1973269804 GeV fm.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ccake_oracle.c")
LIB = os.path.join(HERE, "libccake_oracle.so")
HBARC = 0.1973269804

NVAR = 26
NAUX = 31
(V_X1, V_X2, V_X3, V_U1, V_U2, V_U3, V_S, V_NB, V_NS, V_NQ, V_B,
 V_P11, V_P12, V_P13, V_P22, V_P23, V_P33,
 V_JB1, V_JB2, V_JB3, V_JS1, V_JS2, V_JS3, V_JQ1, V_JQ2, V_JQ3) = range(NVAR)
# kappa_{qq'}/T^2 of the paper's full BSQ diffusion matrix ("BSQ diffusion and
# the beam energy scan"), rows and columns (B, S, Q)
KAPPA_T2_BSQ = ((0.0482, -0.0482, 0.0), (-0.0482, 0.1447, 0.0147), (0.0, 0.0147, 0.0880))
(A_SIGSTAR, A_S, A_NB, A_NS, A_NQ, A_T, A_MUB, A_MUS, A_MUQ, A_P, A_E,
 A_CS2, A_INTABLE, A_GAMMA, A_THETA, A_NNB, A_F1, A_F2, A_F3,
 A_KN_SHEAR, A_REINV_SHEAR, A_KN_BULK, A_REINV_BULK,
 A_DE0, A_DE1, A_DE2, A_DE3, A_DSIG0, A_DSIG1, A_DSIG2, A_DSIG3) = range(NAUX)

EOS_CONFORMAL, EOS_TABLE, EOS_GAS, EOS_MODCONF = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (C11, -O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
            "-shared", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("hyperbolic", ctypes.c_int32),
        ("viscous", ctypes.c_int32), ("ncharge", ctypes.c_int32),
        ("use_cells", ctypes.c_int32), ("nthreads", ctypes.c_int32),
        ("density_mode", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("h", ctypes.c_double), ("eta_over_s", ctypes.c_double),
        ("zeta_peak", ctypes.c_double), ("zeta_Tpeak", ctypes.c_double),
        ("zeta_width", ctypes.c_double), ("taupi_coeff", ctypes.c_double),
        ("tauPi_ratio", ctypes.c_double), ("c_PiPi", ctypes.c_double),
        ("c_Pipi", ctypes.c_double), ("c_pipi", ctypes.c_double),
        ("c_piPi", ctypes.c_double),
        ("nsrc", ctypes.c_int32), ("pad1", ctypes.c_int32),
        ("src", ctypes.c_void_p),
        ("diffusion", ctypes.c_int32), ("pad2", ctypes.c_int32),
        ("kappa_T2", ctypes.c_double * 9), ("tauJ_coeff", ctypes.c_double),
        ("c_JJ", ctypes.c_double), ("c_pisig", ctypes.c_double),
        ("d_JPi", ctypes.c_double * 3),
    ]


class Source(ctypes.Structure):
    """External source (eq. conservation_source): normalised Gaussian of the
    given widths around a centre moving with velocity vel, active for
    t_on <= x0 < t_off, depositing dp^mu/dx0 and dN_q/dx0."""
    _fields_ = [
        ("x0", ctypes.c_double * 3), ("vel", ctypes.c_double * 3), ("width", ctypes.c_double * 3),
        ("t_on", ctypes.c_double), ("t_off", ctypes.c_double),
        ("dpdt", ctypes.c_double * 4), ("dndt", ctypes.c_double * 3),
    ]


def sources(specs):
    """ctypes array of Source from dicts with keys x0, vel, width, t_on,
    t_off, dpdt, dndt (missing vectors are zero)."""
    arr = (Source * max(1, len(specs)))()
    for k, sp in enumerate(specs):
        S = arr[k]
        for name, m in (("x0", 3), ("vel", 3), ("width", 3), ("dpdt", 4), ("dndt", 3)):
            vals = list(sp.get(name, [0.0] * m)) + [0.0] * m
            for i in range(m):
                getattr(S, name)[i] = float(vals[i])
        S.t_on = float(sp.get("t_on", -1e300))
        S.t_off = float(sp.get("t_off", 1e300))
    return arr


class EosC(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("nT", ctypes.c_int32), ("nB", ctypes.c_int32),
        ("nS", ctypes.c_int32), ("nQ", ctypes.c_int32), ("max_iter", ctypes.c_int32),
        ("fstar", ctypes.c_double), ("tol", ctypes.c_double),
        ("lo", ctypes.c_double * 4), ("hi", ctypes.c_double * 4),
        ("cols", ctypes.POINTER(ctypes.c_double)),
        ("A0", ctypes.c_double), ("muq0", ctypes.c_double * 3), ("cq", ctypes.c_double * 3),
        ("inv", ctypes.c_void_p),
    ]


NINV = 9
(I_T, I_MUB, I_MUS, I_MUQ, I_P, I_E, I_CS2, I_KAP, I_TAB) = range(NINV)


class InvC(ctypes.Structure):
    """Offline inverted table: s nodes 10^d (1 + 9 m / P) inside decades
    d0 <= d < d1 plus 10^d1; x_q = n_q / s on uniform grids (ncharge 3)."""
    _fields_ = [
        ("ncharge", ctypes.c_int32), ("d0", ctypes.c_int32), ("d1", ctypes.c_int32),
        ("per_decade", ctypes.c_int32), ("nx", ctypes.c_int32 * 3), ("pad", ctypes.c_int32),
        ("xlo", ctypes.c_double * 3), ("xhi", ctypes.c_double * 3),
        ("val", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.orc_kernel_w.restype = ctypes.c_double
        L.orc_kernel_w.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_kernel_dw_over_r.restype = ctypes.c_double
        L.orc_kernel_dw_over_r.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_pairs.restype = ctypes.c_int64
        L.orc_pairs.argtypes = [ctypes.POINTER(Params), ctypes.c_int64, dp, ctypes.c_int64, ip, ip]
        L.orc_eos_invert.restype = ctypes.c_int
        L.orc_eos_invert.argtypes = [ctypes.POINTER(EosC), ctypes.c_int, ctypes.c_int, ctypes.c_int64, dp, dp, ip]
        L.orc_eos_eval.restype = None
        L.orc_eos_eval.argtypes = [ctypes.POINTER(EosC), ctypes.c_int, ctypes.c_int64, dp, dp]
        L.orc_rhs.restype = ctypes.c_int
        L.orc_rhs.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(EosC), ctypes.c_double,
                              ctypes.c_int64, dp, dp, dp]
        L.orc_heun_step.restype = ctypes.c_int
        L.orc_rhs_targets.restype = ctypes.c_int
        L.orc_rhs_targets.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(EosC), ctypes.c_double,
                                      ctypes.c_int64, dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), dp, dp]
        L.orc_heun_step.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(EosC), ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int64, dp, dp]
        L.orc_init.restype = ctypes.c_int
        L.orc_init.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(EosC), ctypes.c_double,
                               ctypes.c_int64, dp, dp, ctypes.c_int, dp, dp]
        L.orc_totals.restype = None
        L.orc_totals.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(EosC), ctypes.c_double,
                                 ctypes.c_int64, dp, dp]
        L.orc_inv_ns.restype = ctypes.c_int64
        L.orc_inv_ns.argtypes = [ctypes.POINTER(InvC)]
        L.orc_inv_build.restype = ctypes.c_int
        L.orc_inv_build.argtypes = [ctypes.POINTER(EosC), ctypes.POINTER(InvC)]
        L.orc_inv_eval.restype = None
        L.orc_inv_eval.argtypes = [ctypes.POINTER(EosC), ctypes.c_int, ctypes.c_int64, dp, dp, ip]
        assert L.orc_nvar() == NVAR and L.orc_naux() == NAUX and L.orc_ninv() == NINV
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params(dim=2, hyperbolic=True, viscous=False, ncharge=0, h=0.3, eta_over_s=0.0,
           zeta_peak=0.0, zeta_Tpeak_GeV=0.17, zeta_width_GeV=0.02, taupi_coeff=5.0,
           tauPi_ratio=1.0, c_PiPi=1.0, c_Pipi=0.0, c_pipi=4.0 / 3.0, c_piPi=0.0,
           use_cells=None, nthreads=0, density_mode=0, source_specs=None, diffusion=False,
           kappa_T2=KAPPA_T2_BSQ, tauJ_coeff=0.2, c_JJ=0.0, c_pisig=0.0, d_JPi=(0.0, 0.0, 0.0)) -> Params:
    p = Params()
    for q in range(3):
        p.d_JPi[q] = float(d_JPi[q])
    p.c_pisig = c_pisig
    p.diffusion = int(bool(diffusion))
    kT = np.asarray(kappa_T2, dtype=np.float64).reshape(3, 3)
    for i in range(9):
        p.kappa_T2[i] = float(kT.flat[i])
    p.tauJ_coeff, p.c_JJ = tauJ_coeff, c_JJ
    if source_specs:
        arr = sources(source_specs)
        p.nsrc = len(source_specs)
        p.src = ctypes.cast(arr, ctypes.c_void_p)
        p._keep_sources = arr
    p.dim, p.hyperbolic, p.viscous, p.ncharge = dim, int(hyperbolic), int(viscous), ncharge
    p.use_cells = 0 if use_cells is None else int(use_cells)
    p.nthreads = nthreads
    p.density_mode = density_mode
    p.h, p.eta_over_s = h, eta_over_s
    p.zeta_peak = zeta_peak
    p.zeta_Tpeak = zeta_Tpeak_GeV / HBARC
    p.zeta_width = zeta_width_GeV / HBARC
    p.taupi_coeff, p.tauPi_ratio = taupi_coeff, tauPi_ratio
    p.c_PiPi, p.c_Pipi, p.c_pipi, p.c_piPi = c_PiPi, c_Pipi, c_pipi, c_piPi
    return p


@dataclass
class Eos:
    c: EosC
    keep: object = None  # keeps the table buffer alive


def eos_conformal(fstar: float = 11.0) -> Eos:
    e = EosC()
    e.kind, e.fstar, e.tol, e.max_iter = EOS_CONFORMAL, fstar, 1e-13, 60
    return Eos(e)


def eos_gas() -> Eos:
    e = EosC()
    e.kind, e.tol, e.max_iter = EOS_GAS, 1e-13, 60
    return Eos(e)


def eos_modconf(A0, muq0, cq) -> Eos:
    e = EosC()
    e.kind, e.tol, e.max_iter = EOS_MODCONF, 1e-13, 60
    e.A0 = A0
    for q in range(3):
        e.muq0[q] = muq0[q]
        e.cq[q] = cq[q]
    return Eos(e)


def eos_table(cols: np.ndarray, lo_fm, hi_fm, tol=1e-13, max_iter=60) -> Eos:
    """cols: (7, nT, nB, nS, nQ) dimensionless columns; axes in fm^-1."""
    cols = _f64(cols)
    assert cols.ndim == 5 and cols.shape[0] == 7
    e = EosC()
    e.kind = EOS_TABLE
    e.nT, e.nB, e.nS, e.nQ = cols.shape[1:]
    e.tol, e.max_iter = tol, max_iter
    for k in range(4):
        e.lo[k] = lo_fm[k]
        e.hi[k] = hi_fm[k]
    e.cols = _dp(cols)
    return Eos(e, cols)


def eos_inverted(forward: Eos, ncharge: int, d0: int, d1: int, per_decade: int, nx=(2, 2, 2),
                 xlo=(0.0, 0.0, 0.0), xhi=(0.0, 0.0, 0.0)) -> Eos:
    """The forward EoS with an offline inverted table ("EoS inverter",
    offline option) built by the online inverter at every node; stages then
    interpolate it, and invert online only off its grid."""
    v = InvC()
    v.ncharge, v.d0, v.d1, v.per_decade = ncharge, d0, d1, per_decade
    for q in range(3):
        v.nx[q] = int(nx[q]) if ncharge else 1
        v.xlo[q], v.xhi[q] = float(xlo[q]), float(xhi[q])
    ns = lib().orc_inv_ns(ctypes.byref(v))
    shape = (ns, v.nx[0], v.nx[1], v.nx[2], NINV)
    val = np.empty(shape)
    v.val = _dp(val)
    bad = lib().orc_inv_build(ctypes.byref(forward.c), ctypes.byref(v))
    if bad:
        raise RuntimeError(f"offline table: {bad} node inversions did not converge")
    e = EosC.from_buffer_copy(forward.c)
    e.inv = ctypes.cast(ctypes.pointer(v), ctypes.c_void_p)
    out = Eos(e, (forward.keep, val, v))
    out.table = val
    out.grid = v
    return out


def inv_eval(eos: Eos, x4: np.ndarray, fallback: bool = False):
    """Offline lookups at points (s, nB, nS, nQ): rows T, muB, muS, muQ, p, e,
    cs2, kappa, in_table, and whether each point was on the grid."""
    x4 = _f64(x4)
    n = x4.shape[1]
    out = np.empty((NINV, n))
    inside = np.empty(n, np.int32)
    lib().orc_inv_eval(ctypes.byref(eos.c), int(fallback), n, _dp(x4), _dp(out), _ip(inside))
    return out, inside.astype(bool)


def kernel_w(dim, h, r):
    return lib().orc_kernel_w(dim, h, r)


def kernel_dw_over_r(dim, h, r):
    return lib().orc_kernel_dw_over_r(dim, h, r)


def pairs(prm: Params, y: np.ndarray):
    y = _f64(y)
    n = y.shape[1]
    tot = lib().orc_pairs(ctypes.byref(prm), n, _dp(y), 0, None, None)
    a = np.empty(max(tot, 1), np.int32)
    b = np.empty(max(tot, 1), np.int32)
    lib().orc_pairs(ctypes.byref(prm), n, _dp(y), tot, _ip(a), _ip(b))
    return a[:tot], b[:tot]


def eos_invert(eos: Eos, mode: int, ncharge: int, x4: np.ndarray):
    x4 = _f64(x4)
    n = x4.shape[1]
    out = np.empty((4, n))
    it = np.empty(n, np.int32)
    bad = lib().orc_eos_invert(ctypes.byref(eos.c), mode, ncharge, n, _dp(x4), _dp(out), _ip(it))
    return out, it, bad


def eos_eval(eos: Eos, use_table: bool, x4: np.ndarray):
    """Columns p, e, s, nB, nS, nQ, cs2, kappa at points (T, muB, muS, muQ)."""
    x4 = _f64(x4)
    n = x4.shape[1]
    out = np.empty((8, n))
    lib().orc_eos_eval(ctypes.byref(eos.c), int(use_table), n, _dp(x4), _dp(out))
    return out


def init(prm: Params, eos: Eos, t0: float, xi, u, dens_kind: int, dens):
    xi, u, dens = _f64(xi), _f64(u), _f64(dens)
    n = xi.shape[1]
    y = np.zeros((NVAR, n))
    bad = lib().orc_init(ctypes.byref(prm), ctypes.byref(eos.c), t0, n, _dp(xi), _dp(u),
                         dens_kind, _dp(dens), _dp(y))
    if bad:
        raise RuntimeError(f"oracle init: {bad} EoS inversions did not converge")
    return y


def rhs(prm: Params, eos: Eos, t: float, y):
    y = _f64(y)
    n = y.shape[1]
    dy = np.zeros((NVAR, n))
    aux = np.zeros((NAUX, n))
    bad = lib().orc_rhs(ctypes.byref(prm), ctypes.byref(eos.c), t, n, _dp(y), _dp(dy), _dp(aux))
    return dy, aux, bad


def rhs_targets(prm: Params, eos: Eos, t: float, y, targets):
    """Rates and diagnostics at the listed particles only (columns in the
    order of targets)."""
    y = _f64(y)
    n = y.shape[1]
    tg = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    nt = tg.shape[0]
    dy = np.zeros((NVAR, nt))
    aux = np.zeros((NAUX, nt))
    bad = lib().orc_rhs_targets(ctypes.byref(prm), ctypes.byref(eos.c), t, n, _dp(y), nt,
                                tg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(dy), _dp(aux))
    return dy, aux, bad


def heun_step(prm: Params, eos: Eos, t: float, dt: float, y):
    y = _f64(y).copy()
    n = y.shape[1]
    aux = np.zeros((NAUX, n))
    bad = lib().orc_heun_step(ctypes.byref(prm), ctypes.byref(eos.c), t, dt, n, _dp(y), _dp(aux))
    return y, aux, bad


def totals(prm: Params, eos: Eos, t: float, y):
    y = _f64(y)
    out = np.zeros(8)
    lib().orc_totals(ctypes.byref(prm), ctypes.byref(eos.c), t, y.shape[1], _dp(y), _dp(out))
    return out


def evolve(prm: Params, eos: Eos, t0: float, dt: float, nsteps: int, y):
    """nsteps Heun steps from (t0, y); returns (t, y, aux of the last stage)."""
    t = t0
    aux = None
    for _ in range(nsteps):
        y, aux, bad = heun_step(prm, eos, t, dt, y)
        if bad:
            raise RuntimeError(f"oracle: {bad} EoS inversions did not converge at t={t}")
        t += dt
    return t, y, aux


# ---------------------------------------------------------------------------
# Constant-energy-density freeze-out surface ("Freeze-out hypersurface
# construction", eq. efo_surface and eq. fonormal), as a record per particle.
# Reading: a particle crosses e = e_fo in the step [t_{k-1}, t_k] in which its
# energy density, evaluated at the step starts, falls from >= e_fo to < e_fo
# (particles already below e_fo at the first evaluation never cross).  Its
# record holds the crossing time t_fo from linear interpolation of e in x^0
# between the two evaluations, its position moved back from t_k to t_fo
# along its velocity (dx^i/dx^0 = u^i / u^0), and u^i, T, mu_q and the surface
# element d sigma_mu (eq. fonormal with the SPH gradient of e and the time
# derivative from the energy equation, the oracle's A_DSIG rows) at t_k.
FO_ID, FO_T, FO_X1, FO_X2, FO_X3, FO_U1, FO_U2, FO_U3, FO_T_, FO_MUB, FO_MUS, FO_MUQ, \
    FO_DS0, FO_DS1, FO_DS2, FO_DS3 = range(16)
FO_NCOL = 16


def freezeout_records(prm: Params, t_prev, t, e_prev, y, aux, frozen, e_fo):
    """Records (rows of FO_NCOL values) of the particles that cross e_fo
    between an evaluation at t_prev (energy densities e_prev) and one at t
    (state y, diagnostics aux); frozen marks the particles already recorded
    and is updated in place."""
    e = aux[A_E]
    cross = (~frozen) & (e_prev >= e_fo) & (e < e_fo)
    dim = prm.dim
    gam = aux[A_GAMMA]
    recs = np.zeros((int(cross.sum()), FO_NCOL))
    for r, i in enumerate(np.flatnonzero(cross)):
        tfo = t - (t - t_prev) * (e_fo - e[i]) / (e_prev[i] - e[i])
        recs[r, FO_ID] = i
        recs[r, FO_T] = tfo
        for k in range(dim):
            recs[r, FO_X1 + k] = y[V_X1 + k, i] - (t - tfo) * y[V_U1 + k, i] / gam[i]
            recs[r, FO_U1 + k] = y[V_U1 + k, i]
        recs[r, FO_T_] = aux[A_T, i]
        for q in range(3):
            recs[r, FO_MUB + q] = aux[A_MUB + q, i]
        for m in range(4):
            recs[r, FO_DS0 + m] = aux[A_DSIG0 + m, i]
    frozen |= cross
    return recs


def evolve_freezeout(prm: Params, eos: Eos, t0: float, dt: float, nsteps: int, y, e_fo: float):
    """nsteps Heun steps from (t0, y), evaluating the diagnostics at every
    step start t_0 .. t_{nsteps-1} and recording the freeze-out crossings
    between consecutive step starts; returns (t, y, records sorted by
    particle)."""
    n = y.shape[1]
    frozen = np.zeros(n, dtype=bool)
    t, e_prev, t_prev = t0, None, None
    out = []
    for _ in range(nsteps):
        _, aux, bad = rhs(prm, eos, t, y)
        if bad:
            raise RuntimeError(f"oracle: {bad} EoS inversions did not converge at t={t}")
        if e_prev is not None:
            out.append(freezeout_records(prm, t_prev, t, e_prev, y, aux, frozen, e_fo))
        e_prev, t_prev = aux[A_E].copy(), t
        y, _, bad = heun_step(prm, eos, t, dt, y)
        if bad:
            raise RuntimeError(f"oracle: {bad} EoS inversions did not converge at t={t}")
        t += dt
    recs = np.concatenate(out) if out else np.zeros((0, FO_NCOL))
    return t, y, recs[np.argsort(recs[:, FO_ID], kind="stable")]
