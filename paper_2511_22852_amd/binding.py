"""Thin ctypes binding of libccake_hip.so (include/ccake.h).

Argument marshalling only: every step of the SPH stage runs in the library's
HIP kernels.  PyTorch provides the device workspace (a uint8 tensor the
library carves its arrays from) and the HIP stream.  When the shared library
is missing the import of this module fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libccake_hip.so")
HBARC = 0.1973269804

OK, E_ARG, E_HIP, E_NONFINITE, E_EOS_NOCONV, E_CAPACITY, E_STATE, E_NOMEM = range(8)
HOST, DEVICE = 0, 1
CARTESIAN, HYPERBOLIC = 0, 1
FP64, MIXED = 0, 1
DENS_SMOOTHED, DENS_SPECIFIC = 0, 1
INIT_S, INIT_E = 0, 1
NROW = 26
NAUX = 33
(ROW_X1, ROW_X2, ROW_X3, ROW_U1, ROW_U2, ROW_U3, ROW_S, ROW_NB, ROW_NS, ROW_NQ, ROW_B,
 ROW_P11, ROW_P12, ROW_P13, ROW_P22, ROW_P23, ROW_P33,
 ROW_JB1, ROW_JB2, ROW_JB3, ROW_JS1, ROW_JS2, ROW_JS3, ROW_JQ1, ROW_JQ2, ROW_JQ3) = range(NROW)
# kappa_{qq'}/T^2 of the paper's full BSQ diffusion matrix (rows and columns B, S, Q)
KAPPA_T2_BSQ = ((0.0482, -0.0482, 0.0), (-0.0482, 0.1447, 0.0147), (0.0, 0.0147, 0.0880))
(AUX_SIGSTAR, AUX_S, AUX_NB, AUX_NS, AUX_NQ, AUX_T, AUX_MUB, AUX_MUS, AUX_MUQ, AUX_P, AUX_E,
 AUX_CS2, AUX_INTABLE, AUX_GAMMA, AUX_THETA, AUX_NNB, AUX_F1, AUX_F2, AUX_F3, AUX_NEWTON,
 AUX_EOS_EVALS, AUX_KN_SHEAR, AUX_REINV_SHEAR, AUX_KN_BULK, AUX_REINV_BULK, AUX_DE0, AUX_DE1, AUX_DE2,
 AUX_DE3, AUX_DSIG0, AUX_DSIG1, AUX_DSIG2, AUX_DSIG3) = range(NAUX)
FO_NCOL = 16
(FO_ID, FO_T, FO_X1, FO_X2, FO_X3, FO_U1, FO_U2, FO_U3, FO_TEMP, FO_MUB, FO_MUS, FO_MUQ,
 FO_DS0, FO_DS1, FO_DS2, FO_DS3) = range(FO_NCOL)

EXPORTS = [
    "ccake_eos_create_conformal", "ccake_eos_create_gas", "ccake_eos_create_table",
    "ccake_eos_destroy", "ccake_eos_invert", "ccake_eos_invert_noalloc", "ccake_eos_build_inverted",
    "ccake_eos_offline_eval",
    "ccake_workspace_bytes", "ccake_create",
    "ccake_init_particles", "ccake_set_state", "ccake_get_state", "ccake_time", "ccake_step",
    "ccake_check", "ccake_set_sources", "ccake_set_profiling", "ccake_kernel_times", "ccake_rhs", "ccake_read", "ccake_read_fields", "ccake_totals", "ccake_debug_pairs",
    "ccake_debug_pairs_cached", "ccake_set_freezeout", "ccake_freezeout_records",
    "ccake_destroy", "ccake_server_workspace_bytes", "ccake_server_create", "ccake_server_submit", "ccake_server_poll",
    "ccake_server_drain", "ccake_server_release", "ccake_server_stats", "ccake_server_destroy",
    "ccake_last_error",
]


class CcakeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ccake status {status}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("coords", ctypes.c_int32), ("viscous", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("ncharge", ctypes.c_int32), ("density_mode", ctypes.c_int32),
        ("h", ctypes.c_double), ("eta_over_s", ctypes.c_double), ("zeta_peak", ctypes.c_double),
        ("zeta_Tpeak", ctypes.c_double), ("zeta_width", ctypes.c_double),
        ("taupi_coeff", ctypes.c_double), ("tauPi_ratio", ctypes.c_double),
        ("c_PiPi", ctypes.c_double), ("c_Pipi", ctypes.c_double), ("c_pipi", ctypes.c_double),
        ("c_piPi", ctypes.c_double), ("skin", ctypes.c_double),
        ("diffusion", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("kappa_T2", ctypes.c_double * 9), ("tauJ_coeff", ctypes.c_double), ("c_JJ", ctypes.c_double),
        ("c_pisig", ctypes.c_double), ("d_JPi", ctypes.c_double * 3),
    ]


class InvGrid(ctypes.Structure):
    """Grid of the offline inverted EoS table (ccake_inv_grid)."""
    _fields_ = [
        ("ncharge", ctypes.c_int32), ("decade_lo", ctypes.c_int32), ("decade_hi", ctypes.c_int32),
        ("per_decade", ctypes.c_int32), ("nx", ctypes.c_int32 * 3), ("pad", ctypes.c_int32),
        ("x_lo", ctypes.c_double * 3), ("x_hi", ctypes.c_double * 3),
    ]


# rows of ccake_eos_offline_eval
OFFLINE_ROWS = ("T", "muB", "muS", "muQ", "p", "e", "cs2", "kappa", "in_table")


class Source(ctypes.Structure):
    _fields_ = [
        ("x0", ctypes.c_double * 3), ("vel", ctypes.c_double * 3), ("width", ctypes.c_double * 3),
        ("t_on", ctypes.c_double), ("t_off", ctypes.c_double),
        ("dpdt", ctypes.c_double * 4), ("dndt", ctypes.c_double * 3),
    ]


MAX_SOURCES = 16


NEWTON_BINS = 12


class Counters(ctypes.Structure):
    _fields_ = [("nonfinite", ctypes.c_uint32), ("noconv", ctypes.c_uint32), ("backup", ctypes.c_uint32),
                ("newton_iters", ctypes.c_uint32), ("first_bad", ctypes.c_int32),
                ("capacity_err", ctypes.c_uint32), ("in_table", ctypes.c_int64),
                ("newton_hist", ctypes.c_int64 * NEWTON_BINS)]


class EventDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("t0", ctypes.c_double), ("t_end", ctypes.c_double),
                ("xi", ctypes.POINTER(ctypes.c_double)), ("u", ctypes.POINTER(ctypes.c_double)),
                ("dens_kind", ctypes.c_int32), ("dens", ctypes.POINTER(ctypes.c_double)),
                ("user_tag", ctypes.c_int64)]


class EventResult(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("user_tag", ctypes.c_int64), ("n", ctypes.c_int64),
                ("status", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_finish", ctypes.c_double),
                ("state", ctypes.POINTER(ctypes.c_double)), ("totals", ctypes.c_double * 8)]


_lib = None


def lib():
    """Load libccake_hip.so; raises when it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime (same soname); loading torch first makes
        # the library bind to that one instead of bringing a second runtime in
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_22852_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        sig = {
            "ccake_eos_create_conformal": [ctypes.POINTER(vp), dbl],
            "ccake_eos_create_gas": [ctypes.POINTER(vp), i32, dbl],
            "ccake_eos_create_table": [ctypes.POINTER(vp), ip, dp, dp, dp, i32, dbl],
            "ccake_eos_destroy": [vp],
            "ccake_eos_invert": [vp, i32, i32, i64, vp, vp, vp, vp],
            "ccake_eos_invert_noalloc": [vp, i32, i32, i64, vp, vp, vp, vp],
            "ccake_eos_build_inverted": [vp, ctypes.POINTER(InvGrid), vp],
            "ccake_eos_offline_eval": [vp, i32, i64, vp, vp, vp, vp],
            "ccake_workspace_bytes": [ctypes.POINTER(Config), i64, ctypes.POINTER(ctypes.c_size_t)],
            "ccake_create": [ctypes.POINTER(vp), ctypes.POINTER(Config), vp, i64, vp, ctypes.c_size_t, vp],
            "ccake_init_particles": [vp, dbl, vp, vp, i32, vp, i32],
            "ccake_set_state": [vp, dbl, vp, i32],
            "ccake_get_state": [vp, vp, i32],
            "ccake_time": [vp, dp],
            "ccake_step": [vp, dbl, i32],
            "ccake_check": [vp],
            "ccake_set_sources": [vp, i32, ctypes.POINTER(Source)],
            "ccake_set_profiling": [vp, i32],
            "ccake_kernel_times": [vp, dp, ctypes.POINTER(i64)],
            "ccake_rhs": [vp, vp, vp, i32],
            "ccake_read": [vp, i32, vp, i32],
            "ccake_read_fields": [vp, ctypes.c_uint64, ctypes.POINTER(vp), i32],
            "ccake_server_workspace_bytes": [ctypes.POINTER(Config), i64, i32, ctypes.POINTER(ctypes.c_size_t)],
            "ccake_totals": [vp, dp, ctypes.POINTER(Counters)],
            "ccake_debug_pairs": [vp, i64, vp, vp, ctypes.POINTER(i64)],
            "ccake_debug_pairs_cached": [vp, i64, vp, vp, ctypes.POINTER(i64)],
            "ccake_set_freezeout": [vp, dbl],
            "ccake_freezeout_records": [vp, i64, vp, ctypes.POINTER(i64), i32],
            "ccake_destroy": [vp],
            "ccake_server_create": [ctypes.POINTER(vp), ctypes.POINTER(Config), vp, ctypes.c_size_t, i64, i32,
                                    dbl, vp, vp, ctypes.c_size_t],
            "ccake_server_submit": [vp, ctypes.POINTER(EventDesc), ctypes.POINTER(i64)],
            "ccake_server_poll": [vp, ctypes.POINTER(EventResult), i32, ctypes.POINTER(i32)],
            "ccake_server_drain": [vp],
            "ccake_server_release": [vp, ctypes.POINTER(EventResult)],
            "ccake_server_stats": [vp, dp, ctypes.POINTER(i64), ctypes.POINTER(i64), ip],
            "ccake_server_destroy": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int32
        L.ccake_last_error.argtypes = [vp]
        L.ccake_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status, handle=None, what=""):
    if status != OK:
        msg = lib().ccake_last_error(handle).decode() if handle else what
        raise CcakeError(status, msg or what)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def config(dim=2, hyperbolic=True, viscous=False, precision=FP64, ncharge=0, density_mode=DENS_SMOOTHED,
           h=0.3, eta_over_s=0.0, zeta_peak=0.0, zeta_Tpeak_GeV=0.17, zeta_width_GeV=0.02, taupi_coeff=5.0,
           tauPi_ratio=1.0, c_PiPi=1.0, c_Pipi=0.0, c_pipi=4.0 / 3.0, c_piPi=0.0, skin=None,
           diffusion=False, kappa_T2=KAPPA_T2_BSQ, tauJ_coeff=0.2, c_JJ=0.0, c_pisig=0.0, d_JPi=(0.0, 0.0, 0.0)) -> Config:
    c = Config()
    c.diffusion = int(bool(diffusion))
    kT = [float(v) for row in kappa_T2 for v in row]
    assert len(kT) == 9
    for i in range(9):
        c.kappa_T2[i] = kT[i]
    c.tauJ_coeff, c.c_JJ = tauJ_coeff, c_JJ
    c.c_pisig = c_pisig
    for q in range(3):
        c.d_JPi[q] = float(d_JPi[q])
    c.dim, c.coords, c.viscous = dim, HYPERBOLIC if hyperbolic else CARTESIAN, int(viscous)
    c.precision, c.ncharge, c.density_mode = int(precision), ncharge, density_mode
    c.h, c.eta_over_s = h, eta_over_s
    c.zeta_peak, c.zeta_Tpeak, c.zeta_width = zeta_peak, zeta_Tpeak_GeV / HBARC, zeta_width_GeV / HBARC
    c.taupi_coeff, c.tauPi_ratio = taupi_coeff, tauPi_ratio
    c.c_PiPi, c.c_Pipi, c.c_pipi, c.c_piPi = c_PiPi, c_Pipi, c_pipi, c_piPi
    c.skin = 0.1 * h if skin is None else skin
    return c


class Eos:
    """An equation of state on the device (conformal, analytic gas, or 4D table)."""

    def __init__(self, handle):
        self.h = handle

    @classmethod
    def conformal(cls, fstar=11.0):
        h = ctypes.c_void_p()
        _check(lib().ccake_eos_create_conformal(ctypes.byref(h), fstar), what="eos_create_conformal")
        return cls(h)

    @classmethod
    def gas(cls, max_iter=60, tol=1e-13):
        h = ctypes.c_void_p()
        _check(lib().ccake_eos_create_gas(ctypes.byref(h), max_iter, tol), what="eos_create_gas")
        return cls(h)

    @classmethod
    def table(cls, cols, lo_fm, hi_fm, max_iter=60, tol=1e-13):
        cols = _f64(cols)
        n = (ctypes.c_int32 * 4)(*cols.shape[1:])
        lo = (ctypes.c_double * 4)(*lo_fm)
        hi = (ctypes.c_double * 4)(*hi_fm)
        h = ctypes.c_void_p()
        _check(lib().ccake_eos_create_table(ctypes.byref(h), n, lo, hi,
                                            cols.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            max_iter, tol), what="eos_create_table")
        return cls(h)

    def invert(self, mode, ncharge, x4, device="cuda:0", noalloc=False):
        """(s or e, nB, nS, nQ) [4, n] -> (T, muB, muS, muQ) [4, n] and the
        in-table flags; noalloc: through ccake_eos_invert_noalloc."""
        import torch
        x = torch.as_tensor(_f64(x4), device=device).contiguous()
        n = x.shape[1]
        out = torch.empty_like(x)
        it = torch.empty(n, dtype=torch.int32, device=device)
        stream = torch.cuda.current_stream(device)
        fn = lib().ccake_eos_invert_noalloc if noalloc else lib().ccake_eos_invert
        _check(fn(self.h, mode, ncharge, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                  ctypes.c_void_p(it.data_ptr()), ctypes.c_void_p(stream.cuda_stream)), self.h)
        return out.cpu().numpy(), it.cpu().numpy()

    def build_inverted(self, ncharge, decade_lo, decade_hi, per_decade, nx=(2, 2, 2), x_lo=(0.0, 0.0, 0.0),
                       x_hi=(0.0, 0.0, 0.0), device="cuda:0"):
        """Attach the offline inverted table (ccake_eos_build_inverted):
        simulations created afterwards with this EoS interpolate it."""
        import torch
        g = InvGrid()
        g.ncharge, g.decade_lo, g.decade_hi, g.per_decade = ncharge, decade_lo, decade_hi, per_decade
        for q in range(3):
            g.nx[q], g.x_lo[q], g.x_hi[q] = int(nx[q]), float(x_lo[q]), float(x_hi[q])
        stream = torch.cuda.current_stream(device)
        _check(lib().ccake_eos_build_inverted(self.h, ctypes.byref(g), ctypes.c_void_p(stream.cuda_stream)),
               self.h)
        return self

    def offline_eval(self, x4, fallback=False, device="cuda:0"):
        """Offline lookups at (s, nB, nS, nQ) [4, n]: rows OFFLINE_ROWS [9, n]
        and whether each point was on the grid."""
        import torch
        x = torch.as_tensor(_f64(x4), device=device).contiguous()
        n = x.shape[1]
        out = torch.empty((9, n), dtype=torch.float64, device=device)
        inside = torch.empty(n, dtype=torch.int32, device=device)
        stream = torch.cuda.current_stream(device)
        _check(lib().ccake_eos_offline_eval(self.h, int(fallback), n, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(inside.data_ptr()),
                                            ctypes.c_void_p(stream.cuda_stream)), self.h)
        return out.cpu().numpy(), inside.cpu().numpy().astype(bool)

    def close(self):
        if self.h:
            lib().ccake_eos_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sim:
    """One SPH event on the GPU: workspace from torch, its own HIP stream."""

    def __init__(self, cfg: Config, eos: Eos, n: int, device="cuda:0", fill=None):
        """fill: optional byte value written over the whole workspace before
        the simulation is created (results must not depend on it)."""
        import torch
        self.cfg, self.eos, self.n, self.device = cfg, eos, int(n), torch.device(device)
        nb = ctypes.c_size_t()
        _check(lib().ccake_workspace_bytes(ctypes.byref(cfg), self.n, ctypes.byref(nb)), what="workspace_bytes")
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        if fill is not None:
            self.ws.fill_(int(fill))
            torch.cuda.synchronize(self.device)
        base = self.ws.data_ptr()
        self.base = (base + 255) & ~255
        self.stream = torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        _check(lib().ccake_create(ctypes.byref(h), ctypes.byref(cfg), eos.h, self.n, ctypes.c_void_p(self.base),
                                  nb.value, ctypes.c_void_p(self.stream.cuda_stream)), what="ccake_create")
        self.h = h

    # -- state ---------------------------------------------------------------
    def init_particles(self, t0, xi, u, dens_kind, dens):
        xi, u, dens = _f64(xi), _f64(u), _f64(dens)
        _check(lib().ccake_init_particles(self.h, t0, _ptr(xi), _ptr(u), dens_kind, _ptr(dens), HOST), self.h)

    def set_state(self, t, y):
        y = _f64(y)
        assert y.shape == (NROW, self.n)
        _check(lib().ccake_set_state(self.h, t, _ptr(y), HOST), self.h)

    def get_state(self):
        y = np.empty((NROW, self.n))
        _check(lib().ccake_get_state(self.h, _ptr(y), HOST), self.h)
        return y

    @property
    def t(self):
        v = ctypes.c_double()
        _check(lib().ccake_time(self.h, ctypes.byref(v)), self.h)
        return v.value

    # -- evolution -------------------------------------------------------------
    def step(self, dt, nsteps=1):
        _check(lib().ccake_step(self.h, dt, nsteps), self.h)

    def set_sources(self, specs):
        """External sources: dicts with x0, vel, width, t_on, t_off, dpdt, dndt
        (vectors default to zero, the window to always-on)."""
        arr = (Source * max(1, len(specs)))()
        for k, sp in enumerate(specs):
            S = arr[k]
            for name, m in (("x0", 3), ("vel", 3), ("width", 3), ("dpdt", 4), ("dndt", 3)):
                vals = list(sp.get(name, [0.0] * m)) + [0.0] * m
                for i in range(m):
                    getattr(S, name)[i] = float(vals[i])
            S.t_on = float(sp.get("t_on", -1e300))
            S.t_off = float(sp.get("t_off", 1e300))
        _check(lib().ccake_set_sources(self.h, len(specs), arr), self.h)

    def check(self):
        _check(lib().ccake_check(self.h), self.h)

    def synchronize(self):
        self.stream.synchronize()

    def set_profiling(self, enable=True):
        _check(lib().ccake_set_profiling(self.h, int(enable)), self.h)

    def kernel_times(self):
        """(ms, launches) per kernel group: 0 binning, 1 density, 2 EoS, 3 gradients, 4 EoM + update."""
        ms = (ctypes.c_double * 5)()
        nl = (ctypes.c_int64 * 5)()
        _check(lib().ccake_kernel_times(self.h, ms, nl), self.h)
        return list(ms), list(nl)

    # -- evaluation --------------------------------------------------------------
    def rhs(self):
        f = np.empty((NROW, self.n))
        aux = np.empty((NAUX, self.n))
        _check(lib().ccake_rhs(self.h, _ptr(f), _ptr(aux), HOST), self.h)
        return f, aux

    def read(self, field):
        out = np.empty(self.n)
        _check(lib().ccake_read(self.h, field, _ptr(out), HOST), self.h)
        return out

    def read_fields(self, fields):
        """Several diagnostic fields (AUX_*) from one evaluation
        (ccake_read_fields): {field: array}."""
        fields = sorted(set(int(f) for f in fields))
        outs = {f: np.empty(self.n) for f in fields}
        ptrs = (ctypes.c_void_p * NAUX)()
        mask = 0
        for f in fields:
            if 0 <= f < NAUX:
                ptrs[f] = outs[f].ctypes.data
            mask |= 1 << f  # the library rejects fields it does not have
        _check(lib().ccake_read_fields(self.h, mask, ptrs, HOST), self.h)
        return outs

    def totals(self):
        out = np.empty(8)
        cnt = Counters()
        _check(lib().ccake_totals(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(cnt)), self.h)
        return out, cnt

    def pairs(self, cached=False):
        """Neighbour pairs (a, b) sorted by (a, b); cached: the pairs the next
        step's density pass accepts through the last binning's rows
        (ccake_debug_pairs_cached), else those of a fresh binning."""
        import torch
        fn = lib().ccake_debug_pairs_cached if cached else lib().ccake_debug_pairs
        cnt = ctypes.c_int64()
        _check(fn(self.h, 0, None, None, ctypes.byref(cnt)), self.h)
        a = torch.empty(max(cnt.value, 1), dtype=torch.int32, device=self.device)
        b = torch.empty_like(a)
        _check(fn(self.h, cnt.value, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                  ctypes.byref(cnt)), self.h)
        a = a[:cnt.value].cpu().numpy().astype(np.int64)
        b = b[:cnt.value].cpu().numpy().astype(np.int64)
        order = np.lexsort((b, a))
        return a[order], b[order]

    def set_freezeout(self, e_fo):
        """Freeze-out surface at energy density e_fo (fm^-4; 0: off); forgets
        the records so far (ccake_set_freezeout)."""
        _check(lib().ccake_set_freezeout(self.h, float(e_fo)), self.h)

    def freezeout_records(self):
        """Records [count][FO_NCOL] (ccake_freezeout_records), sorted by
        particle."""
        cnt = ctypes.c_int64()
        _check(lib().ccake_freezeout_records(self.h, 0, None, ctypes.byref(cnt), HOST), self.h)
        out = np.empty((max(cnt.value, 1), FO_NCOL))
        _check(lib().ccake_freezeout_records(self.h, cnt.value, _ptr(out), ctypes.byref(cnt), HOST), self.h)
        out = out[:cnt.value]
        return out[np.argsort(out[:, FO_ID], kind="stable")]

    def close(self):
        if getattr(self, "h", None):
            lib().ccake_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching serving loop (ccake_server_*): events are submitted
    as they arrive, admitted by device footprint, stepped together, returned
    when they reach their end time."""

    def __init__(self, cfg: Config, eos: Eos, budget_bytes: int, max_particles: int, max_events: int, dt: float,
                 device="cuda:0", own_arena=False):
        """own_arena: let the server allocate its arena (no caller workspace)."""
        import torch
        self.cfg, self.eos, self.device = cfg, eos, torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        # the arena is a torch tensor the server borrows
        nb = ctypes.c_size_t()
        _check(lib().ccake_server_workspace_bytes(ctypes.byref(cfg), int(max_particles), int(max_events),
                                                  ctypes.byref(nb)), what="ccake_server_workspace_bytes")
        self.ws, base = None, 0
        if not own_arena:
            self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
            base = (self.ws.data_ptr() + 255) & ~255
        h = ctypes.c_void_p()
        _check(lib().ccake_server_create(ctypes.byref(h), ctypes.byref(cfg), eos.h, int(budget_bytes),
                                         int(max_particles), int(max_events), dt,
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.c_void_p(base),
                                         nb.value), what="ccake_server_create")
        self.h = h

    def submit(self, t0, t_end, xi, u, dens_kind, dens, tag=0):
        xi, u, dens = _f64(xi), _f64(u), _f64(dens)
        d = EventDesc()
        d.n = xi.shape[1]
        d.t0, d.t_end = t0, t_end
        dp = ctypes.POINTER(ctypes.c_double)
        d.xi, d.u, d.dens = xi.ctypes.data_as(dp), u.ctypes.data_as(dp), dens.ctypes.data_as(dp)
        d.dens_kind, d.user_tag = dens_kind, tag
        t = ctypes.c_int64()
        _check(lib().ccake_server_submit(self.h, ctypes.byref(d), ctypes.byref(t)), self.h)
        return t.value

    def poll(self, cap=64):
        res = (EventResult * cap)()
        cnt = ctypes.c_int32()
        _check(lib().ccake_server_poll(self.h, res, cap, ctypes.byref(cnt)), self.h)
        out = []
        for k in range(cnt.value):
            r = res[k]
            state = np.ctypeslib.as_array(r.state, shape=(NROW * r.n,)).reshape(NROW, r.n).copy()
            out.append(dict(ticket=r.ticket, tag=r.user_tag, n=r.n, status=r.status, steps=r.steps,
                            t_submit=r.t_submit, t_admit=r.t_admit, t_finish=r.t_finish, state=state,
                            totals=list(r.totals)))
            lib().ccake_server_release(self.h, ctypes.byref(r))
        return out

    def drain(self):
        _check(lib().ccake_server_drain(self.h), self.h)

    def stats(self):
        now, steps, ps, res = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib().ccake_server_stats(self.h, ctypes.byref(now), ctypes.byref(steps), ctypes.byref(ps),
                                        ctypes.byref(res)), self.h)
        return dict(now=now.value, steps=steps.value, particle_steps=ps.value, resident=res.value)

    def close(self):
        if getattr(self, "h", None):
            lib().ccake_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
