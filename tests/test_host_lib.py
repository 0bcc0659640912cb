"""CPU tests of libaxpic.so's host side: it loads, exports every symbol the
header declares, rejects invalid arguments before any launch, and its
energy-sampler tables reproduce the oracle's exact quantiles."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2604_24627_amd import axpic as B
from paper_2604_24627_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "axpic.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(axpic_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = B.load()
    syms = header_symbols()
    assert len(syms) >= 13
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(syms) == sorted(B.EXPORTS)
    assert L.axpic_version() == 1
    assert L.axpic_status_string(-2) == b"output capacity exceeded"


def test_struct_layouts_match_header_sizes():
    # offsets that the C compiler would produce (natural alignment, x86-64)
    assert C.sizeof(B.Grid) == 40
    assert C.sizeof(B.SpeciesC) == 8 * 9 + 8 * 2 + 4 * 2 + 8 * 3 + 8 * 2 + 8 * 2 + 8
    assert B.SpeciesC.off.offset == 136 and B.SpeciesC.n_sorted.offset == 144
    assert B.SpeciesC.p2.offset == 152
    assert B.ParamsC.seed.offset % 8 == 0
    # sizes and offsets printed by a C compiler for include/axpic.h (x86-64)
    assert C.sizeof(B.ParamsC) == 224 and C.sizeof(B.CellsC) == 136
    assert C.sizeof(B.MlpC) == 184
    assert C.sizeof(B.MlpNormC) == 288 and B.MlpNormC.count.offset == 256
    assert B.MlpC.out_lin.offset == 72 and B.MlpC.T_lo.offset == 136


N_TAB, Z0_TAB, Z1_TAB = 3072, -18.0, 36.0


def _hermite_z(tab, z):
    N = N_TAB
    h = (Z1_TAB - Z0_TAB) / N
    t = (z - Z0_TAB) / h
    j = np.clip(np.floor(t).astype(int), 0, N - 1)
    f = t - j
    y0, y1 = tab[j], tab[j + 1]
    m0, m1 = tab[N + 1 + j] * h, tab[N + 2 + j] * h
    y = (2 * f ** 3 - 3 * f ** 2 + 1) * y0 + (f ** 3 - 2 * f ** 2 + f) * m0 + \
        (-2 * f ** 3 + 3 * f ** 2) * y1 + (f ** 3 - f ** 2) * m1
    return np.exp(y)


@pytest.mark.parametrize("which,k", [(0, 0.0), (1, 1.7), (1, 2.3)])
def test_sampler_tables_match_exact_quantiles(which, k):
    L = B.load()
    tab = np.zeros(2 * (N_TAB + 1))
    B.check(L.axpic_sampler_table(which, k, tab.ctypes.data_as(C.c_void_p)), "table")
    rng = np.random.default_rng(11)
    a = rng.integers(0, 2 ** 32, 400, dtype=np.uint64)
    u = np.array([O.u24(int(v)) for v in a] + [2 ** -24, 1 - 2 ** -24, 0.5])
    got = _hermite_z(tab, np.log(u) - np.log1p(-u))
    ref = np.array([O.compton_x(v) if which == 0 else O.gamma_x(k, v) for v in u])
    assert np.max(np.abs(got / ref - 1)) < 2e-8
    # the upper half of the grid (cut spectra of massive axions): by tail probability
    z = np.linspace(18.0, 35.5, 41)
    q = np.exp(-z) / (1.0 + np.exp(-z))
    got = _hermite_z(tab, z)
    ref = np.array([O.compton_x_tail(v) if which == 0 else O.gamma_x_tail(k, v) for v in q])
    assert np.max(np.abs(got / ref - 1)) < 2e-8


def test_invalid_arguments_rejected_on_host():
    L = B.load()
    g = B.make_grid(dict(ndim=4, n=(4, 1, 1), dx=0.2, dt=0.1, omega0=1e17))
    sp = B.SpeciesC()
    assert L.axpic_bin_cells(B.ref(g), B.ref(sp), 1, 0.0, None) == -1
    g = B.make_grid(dict(ndim=1, n=(4, 2, 1), dx=0.2, dt=0.1, omega0=1e17))   # n[1] != 1 in 1D
    assert L.axpic_bin_cells(B.ref(g), B.ref(sp), 1, 0.0, None) == -1
    g = B.make_grid(dict(ndim=1, n=(4, 1, 1), dx=0.2, dt=0.1, omega0=1e17))
    sp.n, sp.capacity = 10, 5                                                   # n > capacity
    assert L.axpic_bin_cells(B.ref(g), B.ref(sp), 1, 0.0, None) == -1
    prm = B.make_params(I.Params(lambda_cap=0.0))                               # cap <= 0
    cells = B.CellsC()
    st = np.zeros(4, np.int64)
    assert L.axpic_sample_emit(B.ref(g), B.ref(cells), B.ref(prm), B.ref(sp), 1, None, 0, 0,
                               B.ref(sp), None, None, None, st.ctypes.data, None, 0, None,
                               None) == -1
    prm = B.make_params(I.Params(r_relax=1.5))
    assert L.axpic_feedback(B.ref(g), B.ref(cells), B.ref(prm), B.ref(sp), None, None, None,
                            None, None, 0, None, None) == -1
    assert L.axpic_sampler_table(2, 0.0, None) == -1


def test_table_entries_reject_invalid_arguments_on_host():
    L = B.load()
    g = B.make_grid(dict(ndim=1, n=(4, 1, 1), dx=0.2, dt=0.1, omega0=1e17))
    cells = B.CellsC()
    cells.ncell = 4
    prm = B.make_params(I.Params())
    net = B.MlpC()
    tab = np.zeros(4 * 2 * 16, np.float32)
    net.x_lo, net.x_hi = 0.01, 100.0
    def mt(channel, nodes, lo, hi):
        return L.axpic_mlp_table(B.ref(g), B.ref(cells), B.ref(prm), channel, B.ref(net), nodes,
                                 lo, hi, tab.ctypes.data, None)
    assert mt(B.PRIMAKOFF, 16, 0.05, 30.0) == -1    # no network blob
    net.blob = tab.ctypes.data          # never dereferenced: every call below is rejected first
    for nodes in (3, B.TAB_MAX_NODES + 1):
        assert mt(B.PRIMAKOFF, nodes, 0.05, 30.0) == -1
    assert mt(0, 16, 0.05, 30.0) == -1                # no slot requested
    assert mt(B.PRIMAKOFF, 16, 0.005, 30.0) == -1     # below the training range
    assert mt(B.PRIMAKOFF, 16, 0.05, 200.0) == -1     # above it
    assert mt(B.PRIMAKOFF, 16, 30.0, 0.05) == -1
    sp = B.SpeciesC()
    sp.kind, sp.n = B.PHOTON, 0
    assert L.axpic_rates_table(B.ref(g), B.ref(cells), B.ref(prm), B.ref(sp), B.PRIMAKOFF, 16,
                               0.01, 100.0, None, None, None, None) == -1   # no table
    assert L.axpic_rates_table(B.ref(g), B.ref(cells), B.ref(prm), B.ref(sp), B.PRIMAKOFF, 16,
                               100.0, 0.01, tab.ctypes.data, None, None, None) == -1
    assert L.axpic_rates_table(B.ref(g), B.ref(cells), B.ref(prm), B.ref(sp), B.PRIMAKOFF, 2,
                               0.01, 100.0, tab.ctypes.data, None, None, None) == -1


def test_allocation_free_diag_rejects_species_beyond_its_scratch_on_host():
    """axpic_diag_noalloc holds its partial sums in a static device array of 2^18
    blocks of 1024 particles: a larger species is refused before any HIP call (the
    array pointers below are host memory and are never dereferenced)."""
    L = B.load()
    buf = np.zeros(4, np.float32)
    out = np.zeros(2)
    sp = B.SpeciesC()
    for d in range(3):
        sp.p[d] = buf.ctypes.data
    sp.w, sp.cell = buf.ctypes.data, buf.ctypes.data
    sp.dtype, sp.kind = B.F32, B.AXION
    sp.n = sp.capacity = sp.n_implicit = (1 << 28) + 1
    assert L.axpic_diag_noalloc(B.ref(sp), 0.0, out.ctypes.data, None) == -6
    assert L.axpic_status_string(-6).startswith(b"input exceeds the static scratch")
    assert L.axpic_diag_noalloc(B.ref(sp), -1.0, out.ctypes.data, None) == -1
    assert L.axpic_diag_noalloc(B.ref(sp), 0.0, None, None) == -1


def test_sort_rejects_invalid_arguments_on_host():
    """axpic_sort_cells: a path outside the three or a short workspace are refused before
    any launch."""
    L = B.load()
    g = B.make_grid(dict(ndim=2, n=(8, 6, 1), dx=0.2, dt=0.1, omega0=1e17))
    fake = 1 << 20                       # never dereferenced: the call returns first
    sp, out = B.SpeciesC(), B.SpeciesC()
    for s, a in ((sp, fake), (out, fake + 64)):
        s.x[0] = s.x[1] = s.p[0] = s.p[1] = s.p[2] = s.w = s.id = s.cell = a
        s.n, s.capacity = 10, 10
    st = np.zeros(4, np.int64)
    need = L.axpic_sort_ws_bytes(B.ref(g), 10)
    assert need > 0
    for path in (3, -1):
        assert L.axpic_sort_cells(B.ref(g), B.ref(sp), path, B.ref(out), None, st.ctypes.data,
                                  fake, need, None, None) == -1
    assert L.axpic_sort_cells(B.ref(g), B.ref(sp), 0, B.ref(out), None, st.ctypes.data, fake,
                              need - 1, None, None) == -1


def test_fill_p2_rejects_invalid_arguments_on_host():
    """axpic_fill_p2: no cache, no momenta, or a start outside [0, n] are refused before
    any launch; a start at n launches nothing."""
    L = B.load()
    fake = 1 << 20                       # never dereferenced: the call returns first
    sp = B.SpeciesC()
    sp.x[0] = sp.p[0] = sp.p[1] = sp.p[2] = sp.w = sp.id = sp.cell = fake
    sp.n, sp.capacity, sp.kind = 10, 10, B.PHOTON
    assert L.axpic_fill_p2(B.ref(sp), 0, None) == -1              # no cache
    sp.p2 = fake + 64
    for start in (-1, 11):
        assert L.axpic_fill_p2(B.ref(sp), start, None) == -1
    assert L.axpic_fill_p2(B.ref(sp), 10, None) == 0              # nothing to fill
    sp.p[1] = None
    assert L.axpic_fill_p2(B.ref(sp), 0, None) == -1              # no momenta
