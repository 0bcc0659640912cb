"""FP64 CPU oracle of the axion Monte-Carlo operators -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP product path never loads it and
shares no code with it (the only common module is the seeded input generator,
which holds none of the method's arithmetic).

The arithmetic lives in ``axpic_oracle.c`` (plain C, FP64, built by
``oracle/build.py``); this module marshals numpy arrays into it and drives a
whole time step in the order the method prescribes (every operator acts on the
population present at the start of the step; feedback is applied last).
"""
from __future__ import annotations

import ctypes as C
import os
import math
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# statistics slots (mirrors the enum in axpic_oracle.h)
ST_NAMES = ["events_P", "events_C", "events_B", "num_P", "num_C", "num_B", "en_P", "en_C", "en_B",
            "abs_num", "abs_en", "ag_events", "ag_num", "ag_en", "capped", "overdepleted",
            "cold_cells", "clamped_cells", "unapplied_E", "abs_events"]
ST = {n: i for i, n in enumerate(ST_NAMES)}
ST_COUNT = len(ST_NAMES)

ME_KEV = 510.99895000


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    _lib = C.CDLL(_LIB_PATH)
    _declare(_lib)
    return _lib


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 3), ("dx", C.c_double),
                ("dt", C.c_double), ("omega0", C.c_double)]


class ParamsC(C.Structure):
    _fields_ = [("g_agg_GeV", C.c_double), ("g_ae", C.c_double),
                ("channels", C.c_int32), ("inverse", C.c_int32),
                ("w_a", C.c_double), ("wa_mul", C.c_double * 3), ("w_gamma_prod", C.c_double),
                ("lambda_cap", C.c_double), ("boost", C.c_double),
                ("eq_stats", C.c_int32), ("kappa_mode", C.c_int32),
                ("kappa_fixed_keV", C.c_double), ("prim_targets", C.c_int32),
                ("prim_inv_ratio", C.c_double), ("brems_ee", C.c_int32),
                ("brems_k", C.c_double), ("brems_theta", C.c_double),
                ("absorb_mode", C.c_int32), ("quasi_neutral", C.c_int32),
                ("T_mode", C.c_int32), ("feedback", C.c_int32),
                ("r_relax", C.c_double), ("T_floor_keV", C.c_double), ("T_ceil_keV", C.c_double),
                ("seed", C.c_uint64), ("hist_lo_keV", C.c_double), ("hist_hi_keV", C.c_double),
                ("hist_nbins", C.c_int32), ("hist_log", C.c_int32), ("m_a_keV", C.c_double),
                ("light_mode", C.c_int32)]


class Species(C.Structure):
    _fields_ = [("x", C.c_void_p * 3), ("p", C.c_void_p * 3), ("w", C.c_void_p),
                ("id", C.c_void_p), ("cell", C.c_void_p), ("n", C.c_int64)]


class Products(C.Structure):
    _fields_ = [("x", C.c_void_p * 3), ("p", C.c_void_p * 3), ("w", C.c_void_p),
                ("id", C.c_void_p), ("cell", C.c_void_p), ("parent", C.c_void_p),
                ("chan", C.c_void_p), ("cap", C.c_int64)]


CELL_FIELDS = ["T", "n_e", "n_e_dep", "nZ", "nZ2", "rho", "XH", "kappa2", "G_P0", "G_C", "G_B",
               "Q_C", "Q_B", "meanE_C", "meanE_B"]
CELL_DTYPE = np.dtype([(f, np.float64) for f in CELL_FIELDS])

_P = C.c_void_p
_D = C.c_double


def _declare(L):
    L.or_const.restype = _D; L.or_const.argtypes = [C.c_int]
    L.or_num_threads.restype = C.c_int32
    L.or_set_num_threads.restype = None; L.or_set_num_threads.argtypes = [C.c_int32]
    L.or_philox4x32_10.argtypes = [_P, _P, _P]
    L.or_draw.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _P]
    L.or_u53.restype = _D; L.or_u53.argtypes = [C.c_uint32, C.c_uint32]
    L.or_u24.restype = _D; L.or_u24.argtypes = [C.c_uint32]
    L.or_poisson.restype = C.c_int32; L.or_poisson.argtypes = [_D, _D]
    L.or_poisson_batch.argtypes = [_P, _P, _P, C.c_int64]
    L.or_F.restype = _D; L.or_F.argtypes = [_D]
    L.or_cell_state.argtypes = [_P, _P, C.c_int64, _P, _P, C.c_int32, _P, _P, _P, _P]
    L.or_gamma_prim.restype = _D; L.or_gamma_prim.argtypes = [_P, _P, _D]
    L.or_gamma_abs.restype = _D; L.or_gamma_abs.argtypes = [_P, _P, _D, _P]
    L.or_dt_phys.restype = _D; L.or_dt_phys.argtypes = [_P]
    L.or_V_cell.restype = _D; L.or_V_cell.argtypes = [_P]
    for f in ("or_compton_cdf", "or_compton_ccdf", "or_compton_x"):
        getattr(L, f).restype = _D; getattr(L, f).argtypes = [_D]
    L.or_gammainc_P.restype = _D; L.or_gammainc_P.argtypes = [_D, _D]
    L.or_gammainc_Q.restype = _D; L.or_gammainc_Q.argtypes = [_D, _D]
    L.or_gamma_x.restype = _D; L.or_gamma_x.argtypes = [_D, _D]
    L.or_hist_bin.restype = C.c_int32; L.or_hist_bin.argtypes = [_P, _D]
    L.or_deposit.argtypes = [_P, C.c_int64, _D, _P]
    L.or_emit_primakoff.restype = C.c_int64
    L.or_emit_primakoff.argtypes = [_P, _P, _P, _P, _P, C.c_int64, C.c_uint64, _P, _P, _P, _P, _P]
    L.or_emit_thermal.restype = C.c_int64
    L.or_emit_thermal.argtypes = [_P, _P, _P, _P, _P, C.c_int64, C.c_uint64, _P, _P, _P, _P, _P, _P]
    L.or_emit_thermal_cells.restype = C.c_int64
    L.or_emit_thermal_cells.argtypes = [_P, _P, _P, _P, _P, C.c_int64, _P, _P, C.c_int64,
                                        C.c_uint64, _P, _P, _P, _P, _P, _P]
    L.or_absorb.restype = C.c_int64
    L.or_absorb.argtypes = [_P, _P, _P, _P, _P, _P, C.c_int64, C.c_uint64, _P, _P, _P, _P, _P,
                            _P, _P]
    L.or_feedback.argtypes = [_P, _P, C.c_int64, _P, _P, _P, _P, _P, _P]
    L.or_push.argtypes = [_P, _P, C.c_int32, C.c_double]
    for f in ("or_F_mass", "or_F_mass_quad"):
        getattr(L, f).restype = _D; getattr(L, f).argtypes = [_D, _D, _D]
    L.or_gamma_conv.restype = _D; L.or_gamma_conv.argtypes = [_P, _P, _D]
    L.or_axion_energy.restype = _D; L.or_axion_energy.argtypes = [_P, _D]
    L.or_compton_x_above.restype = _D; L.or_compton_x_above.argtypes = [_D, _D]
    L.or_gamma_x_above.restype = _D; L.or_gamma_x_above.argtypes = [_D, _D, _D]
    L.or_equilibrium.argtypes = [_P, _P, _P, C.c_int64, _P, _D, _P]
    L.or_sort_cells.restype = C.c_int64; L.or_sort_cells.argtypes = [_P, C.c_int64, _P]
    L.or_compton_x_tail.restype = _D; L.or_compton_x_tail.argtypes = [_D]
    L.or_gamma_x_tail.restype = _D; L.or_gamma_x_tail.argtypes = [_D, _D]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _ref(s):
    return C.byref(s)


# ---------------------------------------------------------------------------
# Scalar helpers
# ---------------------------------------------------------------------------

def num_threads() -> int:
    return int(load().or_num_threads())


def set_num_threads(n: int) -> None:
    load().or_set_num_threads(int(n))


def const(i: int) -> float:
    return load().or_const(i)


def philox(ctr, key):
    L = load()
    c = np.asarray(ctr, dtype=np.uint32); k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    L.or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw(seed, pid, step, stream, block):
    out = np.zeros(4, dtype=np.uint32)
    load().or_draw(seed, pid, step, stream, block, _ptr(out))
    return out


def u53(a, b):
    return load().or_u53(int(a), int(b))


def u24(a):
    return load().or_u24(int(a))


def poisson(lam, u):
    return load().or_poisson(float(lam), float(u))


def poisson_batch(lam, u):
    lam = np.ascontiguousarray(lam, dtype=np.float64); u = np.ascontiguousarray(u, dtype=np.float64)
    k = np.zeros(lam.size, dtype=np.int32)
    load().or_poisson_batch(_ptr(lam), _ptr(u), _ptr(k), lam.size)
    return k


def F(s):
    return load().or_F(float(s))


def compton_cdf(X):
    return load().or_compton_cdf(float(X))


def compton_ccdf(X):
    return load().or_compton_ccdf(float(X))


def compton_x(u):
    return load().or_compton_x(float(u))


def gammainc_P(a, y):
    return load().or_gammainc_P(float(a), float(y))


def gammainc_Q(a, y):
    return load().or_gammainc_Q(float(a), float(y))


def gamma_x(k, u):
    return load().or_gamma_x(float(k), float(u))


def make_grid(g: Dict) -> Grid:
    G = Grid()
    G.ndim = g["ndim"]
    for d in range(3):
        G.n[d] = g["n"][d]
    G.dx = g["dx"]; G.dt = g["dt"]; G.omega0 = g["omega0"]
    return G


def make_params(p) -> ParamsC:
    d = p if isinstance(p, dict) else p.as_dict()
    P = ParamsC()
    for name, _ in ParamsC._fields_:
        v = d[name]
        if name == "wa_mul":
            for i in range(3):
                P.wa_mul[i] = v[i]
        else:
            setattr(P, name, v)
    return P


def dt_phys(grid: Dict) -> float:
    return load().or_dt_phys(_ref(make_grid(grid)))


def V_cell(grid: Dict) -> float:
    return load().or_V_cell(_ref(make_grid(grid)))


def hist_bin(params, E_keV) -> int:
    P = make_params(params)
    return load().or_hist_bin(_ref(P), float(E_keV))


# ---------------------------------------------------------------------------
# Species (FP64, physical weights) and products
# ---------------------------------------------------------------------------

class OSpecies:
    """FP64 SoA with physical weights."""

    def __init__(self, x, p, w, pid, cell):
        self.x = np.ascontiguousarray(x, dtype=np.float64).reshape(3, -1).copy()
        n = self.x.shape[1]
        self.p = (np.zeros((3, n)) if p is None
                  else np.ascontiguousarray(p, dtype=np.float64).reshape(3, -1).copy())
        self.w = np.ascontiguousarray(w, dtype=np.float64).copy()
        self.id = np.ascontiguousarray(pid, dtype=np.uint64).copy()
        self.cell = np.ascontiguousarray(cell, dtype=np.int32).copy()

    @property
    def n(self):
        return self.w.size

    @staticmethod
    def empty():
        return OSpecies(np.zeros((3, 0)), np.zeros((3, 0)), np.zeros(0), np.zeros(0, np.uint64),
                        np.zeros(0, np.int32))

    @staticmethod
    def from_input(sp: Dict):
        return OSpecies(sp["x"], sp["p"], sp["w"].astype(np.float64) * sp["w_ref"], sp["id"],
                        sp["cell"])

    def struct(self) -> Species:
        S = Species()
        for d in range(3):
            S.x[d] = self.x[d].ctypes.data
            S.p[d] = self.p[d].ctypes.data
        S.w = self.w.ctypes.data; S.id = self.id.ctypes.data; S.cell = self.cell.ctypes.data
        S.n = self.n
        return S

    def append(self, prod: "OProducts", count: int):
        self.x = np.concatenate([self.x, prod.x[:, :count]], axis=1)
        self.p = np.concatenate([self.p, prod.p[:, :count]], axis=1)
        self.w = np.concatenate([self.w, prod.w[:count]])
        self.id = np.concatenate([self.id, prod.id[:count]])
        self.cell = np.concatenate([self.cell, prod.cell[:count]])

    def sort_cells(self, ncell: int) -> np.ndarray:
        """Canonical order (or_sort_cells): stable counting sort by cell, particles of zero
        weight dropped; returns the cell offsets [ncell + 1]."""
        off = np.zeros(ncell + 1, np.int64)
        S = self.struct()
        m = load().or_sort_cells(_ref(S), ncell, _ptr(off))
        self.x = np.ascontiguousarray(self.x[:, :m]); self.p = np.ascontiguousarray(self.p[:, :m])
        self.w = self.w[:m].copy(); self.id = self.id[:m].copy(); self.cell = self.cell[:m].copy()
        return off

    def compact(self):
        keep = self.w > 0.0
        self.x = np.ascontiguousarray(self.x[:, keep]); self.p = np.ascontiguousarray(self.p[:, keep])
        self.w = self.w[keep]; self.id = self.id[keep]; self.cell = self.cell[keep]

    def copy(self):
        return OSpecies(self.x, self.p, self.w, self.id, self.cell)


class OProducts:
    def __init__(self, cap: int):
        cap = max(int(cap), 1)
        self.x = np.zeros((3, cap)); self.p = np.zeros((3, cap)); self.w = np.zeros(cap)
        self.id = np.zeros(cap, np.uint64); self.cell = np.zeros(cap, np.int32)
        self.parent = np.zeros(cap, np.int64); self.chan = np.zeros(cap, np.int32)
        self.cap = int(cap)

    def struct(self) -> Products:
        S = Products()
        for d in range(3):
            S.x[d] = self.x[d].ctypes.data
            S.p[d] = self.p[d].ctypes.data
        S.w = self.w.ctypes.data; S.id = self.id.ctypes.data; S.cell = self.cell.ctypes.data
        S.parent = self.parent.ctypes.data; S.chan = self.chan.ctypes.data
        S.cap = self.cap
        return S

    def trimmed(self, n: int) -> Dict:
        return dict(x=self.x[:, :n].copy(), p=self.p[:, :n].copy(), w=self.w[:n].copy(),
                    id=self.id[:n].copy(), cell=self.cell[:n].copy(),
                    parent=self.parent[:n].copy(), chan=self.chan[:n].copy())


# ---------------------------------------------------------------------------
# Operators
# ---------------------------------------------------------------------------

def deposit(sp: OSpecies, ncell: int, V: float) -> np.ndarray:
    d = np.zeros(ncell)
    S = sp.struct()
    load().or_deposit(_ref(S), ncell, V, _ptr(d))
    return d


def cell_state(grid: Dict, params, T: np.ndarray, dens_e: np.ndarray, dens_ions, Zs, As):
    ncell = T.size
    G = make_grid(grid); P = make_params(params)
    out = np.zeros(ncell, dtype=CELL_DTYPE)
    di = np.ascontiguousarray(np.stack([np.asarray(d, dtype=np.float64) for d in dens_ions]))
    Z = np.ascontiguousarray(Zs, dtype=np.float64); A = np.ascontiguousarray(As, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    de = np.ascontiguousarray(dens_e, dtype=np.float64)
    load().or_cell_state(_ref(G), _ref(P), ncell, _ptr(T), _ptr(de), len(Zs), _ptr(di), _ptr(Z),
                         _ptr(A), _ptr(out))
    return out


def gamma_prim(cell_rec, params, omega_keV):
    P = make_params(params)
    c = np.ascontiguousarray(np.array(cell_rec, dtype=CELL_DTYPE).reshape(1))
    return load().or_gamma_prim(_ptr(c), _ref(P), float(omega_keV))


def gamma_abs(cell_rec, params, E_keV):
    P = make_params(params)
    c = np.ascontiguousarray(np.array(cell_rec, dtype=CELL_DTYPE).reshape(1))
    parts = np.zeros(2)
    tot = load().or_gamma_abs(_ptr(c), _ref(P), float(E_keV), _ptr(parts))
    return tot, parts


def emit_primakoff(grid, params, cells, ph: OSpecies, step, next_id, hist=None, stats=None,
                   lam_in=None):
    L = load(); G = make_grid(grid); P = make_params(params)
    n = ph.n
    lam_out = np.zeros(max(n, 1)); K_out = np.zeros(max(n, 1), np.int32)
    li = None if lam_in is None else np.ascontiguousarray(lam_in, dtype=np.float64)
    S = ph.struct()
    need = -L.or_emit_primakoff(_ref(G), _ref(P), _ptr(cells), _ref(S), _ptr(li), step, next_id,
                                None, None, None, None, None)
    prod = OProducts(need)
    PS = prod.struct()
    got = L.or_emit_primakoff(_ref(G), _ref(P), _ptr(cells), _ref(S), _ptr(li), step, next_id,
                              _ref(PS), _ptr(hist), _ptr(stats), _ptr(lam_out), _ptr(K_out))
    assert got == need, (got, need)
    return prod.trimmed(got), lam_out[:n], K_out[:n]


def emit_thermal(grid, params, cells, el: OSpecies, step, next_id, fb=None, hist=None, stats=None,
                 lam_in=None):
    L = load(); G = make_grid(grid); P = make_params(params)
    n = el.n
    lam_out = np.zeros(max(2 * n, 1)); K_out = np.zeros(max(2 * n, 1), np.int32)
    li = None if lam_in is None else np.ascontiguousarray(lam_in, dtype=np.float64).reshape(-1)
    S = el.struct()
    need = -L.or_emit_thermal(_ref(G), _ref(P), _ptr(cells), _ref(S), _ptr(li), step, next_id,
                              None, None, None, None, None, None)
    prod = OProducts(need)
    PS = prod.struct()
    got = L.or_emit_thermal(_ref(G), _ref(P), _ptr(cells), _ref(S), _ptr(li), step, next_id,
                            _ref(PS), _ptr(fb), _ptr(hist), _ptr(stats), _ptr(lam_out), _ptr(K_out))
    assert got == need, (got, need)
    return prod.trimmed(got), lam_out[:2 * n].reshape(2, n), K_out[:2 * n].reshape(2, n)


def emit_thermal_cells(grid, params, cells, el: OSpecies, off, step, next_id, fb=None, hist=None,
                       stats=None, coef_in=None, W_in=None, counts_only=False):
    """Thermal emission by per-cell superposition (or_emit_thermal_cells).
    Returns (products, Lambda [2, ncell], N [2, ncell]); products is None with
    counts_only (nothing is emitted then)."""
    L = load(); G = make_grid(grid); P = make_params(params)
    off = np.ascontiguousarray(off, dtype=np.int64)
    ncell = off.size - 1
    lam = np.zeros(max(2 * ncell, 1)); N = np.zeros(max(2 * ncell, 1), np.int32)
    ci = None if coef_in is None else np.ascontiguousarray(coef_in, dtype=np.float64).reshape(-1)
    wi = None if W_in is None else np.ascontiguousarray(W_in, dtype=np.float64)
    S = el.struct()
    r = L.or_emit_thermal_cells(_ref(G), _ref(P), _ptr(cells), _ref(S), _ptr(off), ncell, _ptr(ci),
                                _ptr(wi), step, next_id, None, None, None, None, _ptr(lam), _ptr(N))
    if counts_only:
        return None, lam[:2 * ncell].reshape(2, ncell), N[:2 * ncell].reshape(2, ncell)
    prod = OProducts(-r)
    PS = prod.struct()
    got = L.or_emit_thermal_cells(_ref(G), _ref(P), _ptr(cells), _ref(S), _ptr(off), ncell,
                                  _ptr(ci), _ptr(wi), step, next_id, _ref(PS), _ptr(fb), _ptr(hist),
                                  _ptr(stats), _ptr(lam), _ptr(N))
    assert got == -r, (got, r)
    return prod.trimmed(got), lam[:2 * ncell].reshape(2, ncell), N[:2 * ncell].reshape(2, ncell)


def absorb(grid, params, cells, ax: OSpecies, step, next_id, fb=None, stats=None, pabs_in=None,
           lam_in=None):
    L = load(); G = make_grid(grid); P = make_params(params)
    n = ax.n
    pab = np.zeros(max(n, 1)); lam = np.zeros(max(n, 1)); K = np.zeros(max(n, 1), np.int32)
    dead = np.zeros(max(n, 1), np.int32)
    pi = None if pabs_in is None else np.ascontiguousarray(pabs_in, dtype=np.float64)
    li = None if lam_in is None else np.ascontiguousarray(lam_in, dtype=np.float64)
    S = ax.struct()
    need = -L.or_absorb(_ref(G), _ref(P), _ptr(cells), _ref(S), _ptr(pi), _ptr(li), step, next_id,
                        None, None, None, None, None, None, None)
    prod = OProducts(need)
    PS = prod.struct()
    got = L.or_absorb(_ref(G), _ref(P), _ptr(cells), _ref(S), _ptr(pi), _ptr(li), step, next_id,
                      _ref(PS), _ptr(fb), _ptr(stats), _ptr(pab), _ptr(lam), _ptr(K), _ptr(dead))
    assert got == need, (got, need)
    return prod.trimmed(got), pab[:n], lam[:n], K[:n], dead[:n]


def feedback(grid, params, off, el: OSpecies, fb, T, stats=None, moments=None):
    L = load(); G = make_grid(grid); P = make_params(params)
    ncell = T.size
    S = el.struct()
    off = np.ascontiguousarray(off, dtype=np.int64)
    L.or_feedback(_ref(G), _ref(P), ncell, _ptr(off), _ref(S), _ptr(fb), _ptr(T), _ptr(stats),
                  _ptr(moments))


EQ_FIELDS = ("num", "en", "w2", "neq", "ueq", "nfix", "z")


def equilibrium(grid, params, cells, sp: OSpecies, t_steps: float = 0.0) -> Dict:
    """Equilibrium check of the thermal inverse operators (or_equilibrium): per bin of
    the histogram grid (nbins bins, then underflow and overflow) the population's
    number, energy and sum of squared weights, the equilibrium number and energy, the
    Jacobi-recursion content after t_steps steps (t_steps <= 0: its fixed point) and
    the residual z = (num - nfix) / sqrt(w2)."""
    L = load(); G = make_grid(grid); P = make_params(params)
    nbh = P.hist_nbins + 2
    out = np.zeros(7 * nbh)
    c = np.ascontiguousarray(cells)
    S = sp.struct()
    L.or_equilibrium(_ref(G), _ref(P), _ptr(c), c.size, _ref(S), float(t_steps), _ptr(out))
    return {k: out[i * nbh:(i + 1) * nbh].copy() for i, k in enumerate(EQ_FIELDS)}


def push(grid, ax: OSpecies, prec32: bool, m_a_keV: float = 0.0):
    """Ballistic push (axions of mass m_a_keV move at p / sqrt(p^2 + (m/m_e)^2))."""
    L = load(); G = make_grid(grid)
    S = ax.struct()
    L.or_push(_ref(G), _ref(S), 1 if prec32 else 0, float(m_a_keV))


def F_mass(k, p, kappa2):
    return load().or_F_mass(float(k), float(p), float(kappa2))


def F_mass_quad(k, p, kappa2):
    return load().or_F_mass_quad(float(k), float(p), float(kappa2))


def gamma_conv(cell_rec, params, omega_keV):
    P = make_params(params)
    c = np.ascontiguousarray(np.array(cell_rec, dtype=CELL_DTYPE).reshape(1))
    return load().or_gamma_conv(_ptr(c), _ref(P), float(omega_keV))


def compton_x_above(xm, u):
    return load().or_compton_x_above(float(xm), float(u))


def gamma_x_above(k, ym, u):
    return load().or_gamma_x_above(float(k), float(ym), float(u))


def compton_x_tail(q):
    return load().or_compton_x_tail(float(q))


def gamma_x_tail(k, q):
    return load().or_gamma_x_tail(float(k), float(q))


# ---------------------------------------------------------------------------
# Whole step
# ---------------------------------------------------------------------------

class OracleSim:
    """One uniform-grid run, FP64 throughout, physical weights.

    Step order (every operator sees the start-of-step population):
      1. push the axions present at the start of the step, re-index their cells and
         put them in the canonical order (stable by cell, zero weights dropped);
      2. local state of every cell from the deposits and the temperature field;
      3. forward Primakoff on the photons, thermal emission on the electrons;
      4. absorption / a->gamma on the axions present before step 3;
      5. feedback remap of the electrons and temperature update.
    """

    def __init__(self, plasma: Dict, params, prec32: bool = False, compact_every: int = 0,
                 sort: bool = True):
        self.grid = plasma["grid"]
        sp = plasma["species"]
        self.pdict = dict(params if isinstance(params, dict) else params.as_dict())
        if not self.pdict["w_gamma_prod"] > 0.0:
            self.pdict["w_gamma_prod"] = sp["photons"]["w_ref"]
        self.params = self.pdict
        self.el = OSpecies.from_input(sp["electrons"])
        self.ion = OSpecies.from_input(sp["ions"])
        self.ph = OSpecies.from_input(sp["photons"])
        self.ax = OSpecies.empty()
        self.el_off = sp["electrons"]["off"].copy()
        self.Z = [sp["ions"]["Z"]]; self.A = [sp["ions"]["A"]]
        self.T = plasma["T_cell"].astype(np.float64).copy()
        self.ncell = self.T.size
        self.V = V_cell(self.grid)
        self.next_id = int(plasma["next_id"])
        self.prec32 = prec32
        self.compact_every = compact_every
        self.sort = sort            # canonical order of the axions after every push
        self.step_index = 0
        nb = self.pdict["hist_nbins"] + 2
        self.hist = np.zeros(3 * nb)
        self.stats = np.zeros(ST_COUNT)
        self.dens_e = deposit(self.el, self.ncell, self.V)
        self.dens_i = deposit(self.ion, self.ncell, self.V)
        self.fb = np.zeros(self.ncell * 4)
        self.last = {}

    def cells(self):
        return cell_state(self.grid, self.params, self.T, self.dens_e, [self.dens_i], self.Z, self.A)

    def step(self, lam_P=None, lam_T=None, pabs=None, lam_ag=None):
        p = self.pdict
        s = self.step_index
        push(self.grid, self.ax, self.prec32, p["m_a_keV"])
        if self.sort:
            self.ax.sort_cells(self.ncell)
        cells = self.cells()
        self.fb[:] = 0.0
        n_ax0 = self.ax.n
        new_ax = []
        if p["channels"] & 1:
            prod, lam, K = emit_primakoff(self.grid, self.params, cells, self.ph, s, self.next_id,
                                          self.hist, self.stats, lam_in=lam_P)
            self.next_id += prod["w"].size
            new_ax.append(prod)
            self.last["lam_P"] = lam; self.last["K_P"] = K
        if p["channels"] & 6:
            prod, lam, K = emit_thermal(self.grid, self.params, cells, self.el, s, self.next_id,
                                        self.fb, self.hist, self.stats, lam_in=lam_T)
            self.next_id += prod["w"].size
            new_ax.append(prod)
            self.last["lam_T"] = lam; self.last["K_T"] = K
        if p["inverse"] and n_ax0 > 0:
            prod, pab, lam, K, dead = absorb(self.grid, self.params, cells, self.ax, s, self.next_id,
                                             self.fb, self.stats, pabs_in=pabs, lam_in=lam_ag)
            self.next_id += prod["w"].size
            self.last.update(pabs=pab, lam_ag=lam, K_ag=K, dead=dead)
            if prod["w"].size:
                _append_dict(self.ph, prod)
        for prod in new_ax:
            _append_dict(self.ax, prod)
        if p["feedback"] or p["T_mode"] == 2:
            feedback(self.grid, self.params, self.el_off, self.el, self.fb, self.T, self.stats)
        self.step_index += 1
        if self.compact_every and self.step_index % self.compact_every == 0:
            self.ax.compact()
        return cells

    def totals(self):
        mu = self.pdict["m_a_keV"] / ME_KEV
        E = ME_KEV * np.sqrt((self.ax.p ** 2).sum(axis=0) + mu * mu)
        return dict(N_a=float(self.ax.w.sum()), U_a=float((self.ax.w * E).sum()))


def _append_dict(sp: OSpecies, prod: Dict):
    sp.x = np.concatenate([sp.x, prod["x"]], axis=1)
    sp.p = np.concatenate([sp.p, prod["p"]], axis=1)
    sp.w = np.concatenate([sp.w, prod["w"]])
    sp.id = np.concatenate([sp.id, prod["id"]])
    sp.cell = np.concatenate([sp.cell, prod["cell"]])
