"""The FP64 equilibrium check on the GPU (axpic_equilibrium; Sec. II.I, eq. gamma_abs,
the relaxation plateau of Sec. III.E) against the oracle's (needs an MI355X).

Both sides take the same seeded input: a plasma graded in temperature (so that the
cells' equilibrium spectra differ) and a seeded axion population (inputs.make_axions),
ragged against the library's segment of 4096 particles and chunk of 256 cells.
Bars: the population columns (sums of FP64 values) to 1e-12 relative; the reference
columns (bin integrals by different quadrature orders) to 1e-9; the residual z to
1e-8 relative.  The result is bitwise the same on a repeated call.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_2604_24627_amd import inputs as I  # noqa: E402
from paper_2604_24627_amd.sim import AxpicSim  # noqa: E402


def _case(dtype, m, mb, per_cell, n=(23, 13), chan=6):
    p = I.Params(g_agg_GeV=1e-10, g_ae=1e-13, channels=chan, inverse=1, w_a=1e-36, boost=4e33,
                 eq_stats=mb, m_a_keV=m, hist_lo_keV=0.3, hist_hi_keV=25.0, hist_nbins=48,
                 hist_log=1)
    wl = I.Workload("eq", ndim=2, n=n, ppc=16, dtype=dtype, T_keV=1.0, T_keV_hi=5.0, n_e=6e25,
                    n_ref=6e25, params=p)
    pl = I.make_plasma(wl, 2)
    print(f"[equilibrium] n={wl.n} dtype={dtype} m={m} mb={mb} axions/cell={per_cell}",
          flush=True)
    g = AxpicSim(pl, wl.params)
    o = O.OracleSim(pl, wl.params, prec32=(dtype == "f32"))
    axd = I.make_axions(wl, pl, per_cell, seed=31)
    g.load_axions(axd)
    return wl, g, o, axd


def _trim(axd, n):
    """The first n particles of a population dict."""
    N = axd["n"]
    out = {k: (v[..., :n] if isinstance(v, np.ndarray) and v.shape[-1:] == (N,) else v)
           for k, v in axd.items()}
    out["n"] = n
    return out


@pytest.mark.parametrize("dtype,m,mb", [("f32", 0.0, 0), ("f64", 0.0, 1), ("f32", 1.5, 0)])
def test_equilibrium_matches_oracle(dtype, m, mb):
    wl, g, o, axd = _case(dtype, m, mb, per_cell=15.0)
    assert g.ax.n % 4096 != 0 and g.ncell % 256 != 0 and g.ax.n > 4096
    cells = o.cells()
    osp = O.OSpecies.from_input(axd)
    for t in (0.0, 37.0):
        got = g.equilibrium(t_steps=t)
        ref = O.equilibrium(o.grid, o.params, cells, osp, t_steps=t)
        for k in ("num", "en", "w2"):
            np.testing.assert_allclose(got[k], ref[k], rtol=1e-12, atol=0)
        for k in ("neq", "ueq", "nfix"):
            np.testing.assert_allclose(got[k], ref[k], rtol=1e-9,
                                       atol=1e-12 * np.abs(ref[k]).max())
        # z inherits the relative error of num - nfix (this population is far from
        # equilibrium: |z| is large, num and nfix do not cancel)
        np.testing.assert_allclose(got["z"], ref["z"], rtol=1e-8, atol=1e-8 * np.abs(ref["z"]).max())
        assert (got["neq"] > 0).sum() > 30
    again = g.equilibrium(t_steps=37.0)
    for k in got:
        np.testing.assert_array_equal(again[k], got[k])


def test_equilibrium_of_an_empty_population_and_one_segment_exactly():
    wl, g, o, axd = _case("f32", 0.0, 0, per_cell=30.0)
    cells = o.cells()
    empty = _trim(axd, 0)
    g.load_axions(empty)
    assert g.ax.n == 0
    got = g.equilibrium()
    ref = O.equilibrium(o.grid, o.params, cells, O.OSpecies.empty())
    assert np.all(got["num"] == 0) and np.all(got["z"] == 0)
    np.testing.assert_allclose(got["nfix"], ref["nfix"], rtol=1e-9)
    for n in (4096, 4097, 8192):          # one full segment, one particle more, two segments
        sub = _trim(axd, n)
        g.load_axions(sub)
        got = g.equilibrium()
        ref = O.equilibrium(o.grid, o.params, cells, O.OSpecies.from_input(sub))
        for k in ("num", "en", "w2"):
            np.testing.assert_allclose(got[k], ref[k], rtol=1e-12)
