"""ctypes binding of libaxpic.so (include/axpic.h): argument marshalling only.

Every numerical step runs in the HIP kernels of the library; this module
turns torch tensors into device pointers and raises on any non-OK status.
Loading fails loudly when the library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaxpic.so")

F32, F64 = 0, 1
ELECTRON, ION, PHOTON, AXION = 0, 1, 2, 3
PRIMAKOFF, COMPTON, BREMS = 1, 2, 4
MAX_IONS, PREF_N, STATE_N, STATUS_N = 4, 8, 16, 4
FLAG_CAPACITY = 1
FLAG_SKIPPED = 4
SORT_AUTO, SORT_SPARSE, SORT_DENSE = 0, 1, 2
CHAIN_AXIONS, CHAIN_PHOTONS, CHAIN_NEXT_ID, CHAIN_SKIP, CHAIN_AX_START = 0, 1, 2, 3, 4
CHAIN_N = 5
ST_NAMES = ["events_P", "events_C", "events_B", "num_P", "num_C", "num_B", "en_P", "en_C", "en_B",
            "abs_num", "abs_en", "ag_events", "ag_num", "ag_en", "capped", "overdepleted",
            "cold_cells", "clamped_cells", "unapplied_E", "abs_events"]
ST = {n: i for i, n in enumerate(ST_NAMES)}
ST_COUNT = len(ST_NAMES)
STATUS_MSG = {0: "ok", -1: "invalid argument", -2: "capacity", -3: "domain", -4: "device",
              -5: "unsupported", -6: "input exceeds the static scratch"}


class AxpicError(RuntimeError):
    pass


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 3), ("dx", C.c_double),
                ("dt", C.c_double), ("omega0", C.c_double)]


class SpeciesC(C.Structure):
    _fields_ = [("x", C.c_void_p * 3), ("p", C.c_void_p * 3), ("w", C.c_void_p),
                ("id", C.c_void_p), ("cell", C.c_void_p), ("n", C.c_int64),
                ("capacity", C.c_int64), ("dtype", C.c_int32), ("kind", C.c_int32),
                ("w_ref", C.c_double), ("Z", C.c_double), ("A", C.c_double),
                ("id0", C.c_uint64), ("n_implicit", C.c_int64), ("off", C.c_void_p),
                ("n_sorted", C.c_int64), ("p2", C.c_void_p)]


class CellsC(C.Structure):
    _fields_ = [("ncell", C.c_int64), ("T_keV", C.c_void_p), ("dens", C.c_void_p),
                ("state", C.c_void_p), ("pref32", C.c_void_p), ("pref64", C.c_void_p),
                ("nion", C.c_int32), ("Zion", C.c_double * MAX_IONS),
                ("Aion", C.c_double * MAX_IONS), ("w_ref_e", C.c_double), ("w_ref_g", C.c_double)]


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


EXPORTS = ["axpic_status_string", "axpic_version", "axpic_workspace_bytes", "axpic_bin_cells",
           "axpic_deposit", "axpic_cell_state", "axpic_rates", "axpic_sample_emit",
           "axpic_fill_p2",
           "axpic_absorb", "axpic_feedback", "axpic_compact", "axpic_diag",
           "axpic_sampler_table", "axpic_timing_enable", "axpic_timing_only",
           "axpic_timing_read",
           "axpic_stream_copy", "axpic_mlp_blob_bytes", "axpic_mlp_train_ws_bytes",
           "axpic_mlp_pack", "axpic_mlp_forward", "axpic_mlp_loss_grad", "axpic_mlp_adam",
           "axpic_rates_mlp", "axpic_surrogate_samples", "axpic_cell_weights",
           "axpic_sample_emit_cells", "axpic_mlp_table", "axpic_rates_table",
           "axpic_mlp_prepare_ws_bytes", "axpic_mlp_prepare", "axpic_mlp_design",
           "axpic_mlp_batch", "axpic_equilibrium_ws_bytes", "axpic_equilibrium",
           "axpic_diag_noalloc", "axpic_sort_ws_bytes", "axpic_sort_cells"]
EQ_FIELDS = ("num", "en", "w2", "neq", "ueq", "nfix", "z")
MLP_PARAMS = 57888
MLP_BF16, MLP_F32 = 0, 1
MLP_BLOB_BYTES = 112704
TAB_MAX_NODES = 64


class MlpNormC(C.Structure):
    _fields_ = [("lo", C.c_double * 4), ("sc", C.c_double * 4), ("mu", C.c_double * 4),
                ("lin", C.c_double * 16), ("sigma", C.c_double * 4), ("count", C.c_int64 * 4)]


class MlpC(C.Structure):
    _fields_ = [("blob", C.c_void_p), ("feat_lo", C.c_float * 4), ("feat_sc", C.c_float * 4),
                ("out_mu", C.c_float * 4), ("out_sigma", C.c_float * 4),
                ("out_lin", C.c_float * 16),
                ("T_lo", C.c_double), ("T_hi", C.c_double), ("ne_lo", C.c_double),
                ("ne_hi", C.c_double), ("x_lo", C.c_double), ("x_hi", C.c_double)]

_lib = None
_P = C.c_void_p


def load(path: Optional[str] = None):
    """Load libaxpic.so.  torch is imported first so that its HIP runtime is the
    one the library binds to (same SONAME)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise AxpicError(f"{p} is missing: build it with paper_2604_24627_amd/build.py "
                         "(there is no non-HIP fallback)")
    L = C.CDLL(p)
    L.axpic_status_string.restype = C.c_char_p; L.axpic_status_string.argtypes = [C.c_int32]
    L.axpic_version.restype = C.c_int32
    L.axpic_workspace_bytes.restype = C.c_size_t; L.axpic_workspace_bytes.argtypes = [C.c_int64]
    for f, args in [
        ("axpic_bin_cells", [_P, _P, C.c_int32, C.c_double, _P]),
        ("axpic_deposit", [_P, _P, _P, _P, C.c_int32, _P]),
        ("axpic_cell_state", [_P, _P, _P, C.c_double, C.c_double, _P]),
        ("axpic_fill_p2", [_P, C.c_int64, _P]),
        ("axpic_rates", [_P, _P, _P, _P, C.c_int32, _P, _P]),
        ("axpic_sample_emit", [_P, _P, _P, _P, C.c_int32, _P, C.c_int64, C.c_uint64, _P, _P, _P,
                               _P, _P, _P, C.c_size_t, _P, _P]),
        ("axpic_absorb", [_P, _P, _P, _P, _P, _P, C.c_int64, C.c_uint64, _P, _P, _P, _P, _P,
                          C.c_size_t, _P, _P]),
        ("axpic_feedback", [_P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P, _P]),
        ("axpic_compact", [_P, _P, _P, _P, C.c_size_t, _P]),
        ("axpic_diag", [_P, C.c_double, _P, _P, C.c_size_t, _P]),
        ("axpic_sampler_table", [C.c_int32, C.c_double, _P]),
        ("axpic_timing_read", [C.c_char_p, C.c_size_t]),
        ("axpic_stream_copy", [_P, _P, C.c_size_t, _P]),
        ("axpic_mlp_pack", [_P, _P, _P]),
        ("axpic_mlp_forward", [_P, _P, C.c_int64, C.c_int32, _P, C.c_size_t, _P, _P]),
        ("axpic_mlp_loss_grad", [_P, _P, _P, C.c_int64, C.c_int32, _P, C.c_size_t, _P, _P, _P]),
        ("axpic_mlp_adam", [_P, _P, _P, _P, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float,
                            _P]),
        ("axpic_rates_mlp", [_P, _P, _P, _P, C.c_int32, _P, _P, _P, _P]),
        ("axpic_surrogate_samples", [_P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P]),
        ("axpic_cell_weights", [_P, _P, C.c_int64, _P, _P]),
        ("axpic_sample_emit_cells", [_P, _P, _P, _P, _P, _P, C.c_int32, C.c_int64, C.c_uint64,
                                     _P, _P, _P, _P, _P, _P, C.c_size_t, _P, _P]),
        ("axpic_mlp_table", [_P, _P, _P, C.c_int32, _P, C.c_int32, C.c_double, C.c_double, _P,
                             _P]),
        ("axpic_rates_table", [_P, _P, _P, _P, C.c_int32, C.c_int32, C.c_double, C.c_double, _P,
                               _P, _P, _P]),
        ("axpic_mlp_prepare", [_P, _P, _P, C.c_int64, _P, C.c_size_t, _P, _P]),
        ("axpic_mlp_design", [_P, _P, _P, C.c_int64, _P, _P, _P, _P]),
        ("axpic_mlp_batch", [_P, _P, C.c_int64, C.c_int64, C.c_uint64, C.c_int64, _P, _P, _P]),
        ("axpic_equilibrium", [_P, _P, _P, _P, C.c_double, _P, _P, C.c_size_t, _P]),
        ("axpic_diag_noalloc", [_P, C.c_double, _P, _P]),
        ("axpic_sort_cells", [_P, _P, C.c_int32, _P, _P, _P, _P, C.c_size_t, _P, _P]),
    ]:
        fn = getattr(L, f)
        fn.restype = C.c_int32
        fn.argtypes = args
    L.axpic_mlp_blob_bytes.restype = C.c_size_t
    L.axpic_mlp_prepare_ws_bytes.restype = C.c_size_t
    L.axpic_mlp_prepare_ws_bytes.argtypes = []
    L.axpic_mlp_train_ws_bytes.restype = C.c_size_t
    L.axpic_mlp_train_ws_bytes.argtypes = [C.c_int64]
    L.axpic_sort_ws_bytes.restype = C.c_size_t
    L.axpic_sort_ws_bytes.argtypes = [_P, C.c_int64]
    L.axpic_equilibrium_ws_bytes.restype = C.c_size_t
    L.axpic_equilibrium_ws_bytes.argtypes = [C.c_int64, C.c_int64, C.c_int32]
    L.axpic_timing_enable.restype = None
    L.axpic_timing_enable.argtypes = [C.c_int32]
    L.axpic_timing_only.restype = None
    L.axpic_timing_only.argtypes = [C.c_char_p]
    _lib = L
    return L


def timing_read() -> dict:
    """Per-kernel {name: (launches, total_ms)} since the last read."""
    L = load()
    buf = C.create_string_buffer(1 << 16)
    check(L.axpic_timing_read(buf, len(buf)), "timing_read")
    out = {}
    for line in buf.value.decode().splitlines():
        name, calls, ms = line.split()
        out[name] = (int(calls), float(ms))
    return out


def check(rc: int, what: str):
    if rc != 0:
        raise AxpicError(f"{what}: {STATUS_MSG.get(rc, rc)}")


def ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def ref(s):
    return C.byref(s)


def make_grid(g) -> Grid:
    G = Grid()
    G.ndim = g["ndim"]
    for d in range(3):
        G.n[d] = g["n"][d]
    G.dx, G.dt, G.omega0 = g["dx"], g["dt"], g["omega0"]
    return G


def make_params(p) -> ParamsC:
    d = p if isinstance(p, dict) else p.as_dict()
    P = ParamsC()
    for name, _ in ParamsC._fields_:
        v = d[name]
        if name == "wa_mul":
            for i in range(3):
                P.wa_mul[i] = float(v[i])
        else:
            setattr(P, name, v)
    return P


def stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream
