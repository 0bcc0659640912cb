"""The canonical buffer order on the GPU (axpic_sort_cells) against the oracle's
(or_sort_cells): a stable counting sort by cell with the particles of zero weight
dropped.  Bit-exact: every array, the cell offsets and the kept count, for shuffled
inputs (so that the order within a cell is the test of stability), cells holding more
particles than a wavefront, ragged sizes, an empty input and an output that does not
fit; both ways of taking the counts (per run, per block) and the automatic choice
(needs an MI355X)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_2604_24627_amd import inputs as I  # noqa: E402
from paper_2604_24627_amd import axpic as B  # noqa: E402
from paper_2604_24627_amd.sim import AxpicSim, DeviceSpecies  # noqa: E402


def _shuffled(axd, seed):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(axd["n"])
    out = dict(axd)
    for k in ("x", "p"):
        out[k] = np.ascontiguousarray(axd[k][:, perm])
    for k in ("w", "id", "cell"):
        out[k] = np.ascontiguousarray(axd[k][perm])
    return out


def _sort_on_gpu(g, sp_in, cap=None, path=B.SORT_AUTO):
    out = DeviceSpecies(B.AXION, g.dtype, g.ndim, cap or max(sp_in.n, 1), sp_in.w_ref, g.device)
    off = torch.full((g.ncell + 1,), -7, dtype=torch.int64, device="cuda")
    st = torch.zeros(B.STATUS_N, dtype=torch.int64, device="cuda")
    need = int(g.lib.axpic_sort_ws_bytes(B.ref(g.grid), sp_in.n))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    B.check(g.lib.axpic_sort_cells(B.ref(g.grid), B.ref(sp_in.struct()), path,
                                   B.ref(out.struct()), B.ptr(off), B.ptr(st), B.ptr(ws), need,
                                   None, g.sh), "sort_cells")
    torch.cuda.synchronize()
    return out, off.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("path", [B.SORT_SPARSE, B.SORT_DENSE, B.SORT_AUTO])
@pytest.mark.parametrize("dtype,n,per_cell", [("f32", (23, 13), 5.0), ("f64", (23, 13), 5.0),
                                               ("f32", (7, 3), 41.0), ("f32", (37, 29), 0.3),
                                               ("f32", (256, 128), 6.0), ("f64", (3, 2), 2500.0),
                                               ("f32", (2, 1), 6000.0)])
def test_sort_matches_oracle_bit_exact(dtype, n, per_cell, path):
    p = I.Params(w_a=1e-36)
    wl = I.Workload("sort", ndim=2, n=n, ppc=4, dtype=dtype, T_keV=3.0, n_e=6e25, params=p)
    pl = I.make_plasma(wl, 1)
    axd = _shuffled(I.make_axions(wl, pl, per_cell, seed=3, zero_frac=0.1), 8)
    print(f"[sort] n={n} dtype={dtype} particles={axd['n']} path={path}", flush=True)
    g = AxpicSim(pl, wl.params)
    g.load_axions(axd)
    out, off, st = _sort_on_gpu(g, g.ax, path=path)
    osp = O.OSpecies.from_input(axd)
    ooff = osp.sort_cells(g.ncell)
    assert st[2] == osp.n and st[1] == 0 and osp.n < axd["n"]
    out.n = int(st[2])
    got = out.to_numpy()
    np.testing.assert_array_equal(off, ooff)
    np.testing.assert_array_equal(got["id"], osp.id)
    np.testing.assert_array_equal(got["cell"], osp.cell)
    np.testing.assert_array_equal(got["w"].astype(np.float64) * axd["w_ref"], osp.w)
    np.testing.assert_array_equal(got["p"].astype(np.float64), osp.p)
    np.testing.assert_array_equal(got["x"][:2].astype(np.float64), osp.x[:2])
    if per_cell > 64:
        assert np.diff(ooff).max() > 64
    if per_cell > 5000:                 # cells beyond the gather's LDS window of 4096
        assert np.diff(ooff).max() > 4096


def test_sort_of_nothing_and_of_an_output_that_does_not_fit():
    p = I.Params(w_a=1e-36)
    wl = I.Workload("sort", ndim=2, n=(9, 9), ppc=4, dtype="f32", T_keV=3.0, n_e=6e25, params=p)
    pl = I.make_plasma(wl, 1)
    g = AxpicSim(pl, wl.params)
    empty = DeviceSpecies(B.AXION, g.dtype, g.ndim, 4, wl.params.w_a, g.device)
    out, off, st = _sort_on_gpu(g, empty)
    assert st[2] == 0 and st[1] == 0 and np.all(off == 0)
    axd = I.make_axions(wl, pl, 6.0, seed=4, zero_frac=0.0)
    g.load_axions(axd)
    out, off, st = _sort_on_gpu(g, g.ax, cap=axd["n"] - 1)
    assert st[1] & B.FLAG_CAPACITY and st[0] == axd["n"] and st[2] == 0
    assert np.all(off == -7)                    # nothing written


@pytest.mark.parametrize("chained", [True, False])
def test_stepping_with_the_sort_matches_the_oracle(chained):
    """Full steps (forward and inverse channels, T evolved) on both sides, both in the
    canonical order after every push: the axion buffers equal element for element.  Both
    ways of sorting inside a step -- chained (the kept count stays on the device) and
    with the count read back first (as the surrogate's steps do) -- while absorption
    deletes axions, so that every sort drops some."""
    p = I.Params(g_agg_GeV=1e-10, g_ae=1e-13, channels=7, inverse=1, w_a=1e-36, boost=4e33,
                 lambda_cap=1.0)
    wl = I.Workload("sortstep", ndim=2, n=(12, 10), ppc=24, dtype="f64", T_keV=3.0, n_e=6e25,
                    params=p)
    pl = I.make_plasma(wl, 2)
    g = AxpicSim(pl, wl.params)
    g.sort_chained = chained
    o = O.OracleSim(pl, wl.params, prec32=False)
    dropped = 0
    for s in range(6):
        n_before = g.ax.n
        g.step()
        o.step()
        a = g.ax.to_numpy()
        assert g.ax.n == o.ax.n, (s, g.ax.n, o.ax.n)
        np.testing.assert_array_equal(a["id"], o.ax.id)
        np.testing.assert_array_equal(a["cell"], o.ax.cell)
        assert np.all(np.diff(a["cell"][: g.ax.n_sorted]) >= 0)
        assert np.unique(a["id"]).size == g.ax.n
        dropped += n_before - g.ax.n_sorted
    assert g.ax.n > 100
    assert dropped > 0            # some sorts dropped absorbed axions


@pytest.mark.parametrize("per_cell", [12.0, 0.9])
def test_absorption_over_the_sorted_prefix_decides_as_without_offsets(per_cell):
    """Tiles of the cell-ordered prefix stage their cells' prefactors in LDS (up to 256
    cells per 1024 axions; sparser tiles read them directly): the fused absorption and
    a->gamma over a sorted population decide exactly as the same population without
    offsets, and as the rate-fed path."""
    p = I.Params(g_agg_GeV=1e-10, g_ae=1e-13, channels=7, inverse=1, w_a=1e-36, boost=4e33,
                 lambda_cap=1.0)
    wl = I.Workload("sortabs", ndim=2, n=(64, 40), ppc=8, dtype="f32", T_keV=3.0, n_e=6e25,
                    params=p)
    pl = I.make_plasma(wl, 3)
    axd = I.make_axions(wl, pl, per_cell, seed=9, zero_frac=0.05)
    runs = []
    for mode in ("staged", "plain", "fed"):
        g = AxpicSim(pl, wl.params)
        g.load_axions(axd)
        g.sort_axions()
        assert g.ax.off is not None and g.ax.n_sorted == g.ax.n
        if mode == "plain":
            g.ax.off, g.ax.n_sorted = None, 0
        g.step_index = 4
        n = g.ax.n
        if mode == "fed":
            pab = g.rates(g.ax, B.COMPTON | B.BREMS).clone()
            lag = g.rates(g.ax, B.PRIMAKOFF).clone()
            k = g.absorb(n, pabs_in=pab, lam_in=lag)
        else:
            k = g.absorb(n)
        runs.append((k, g.ax.to_numpy(), g.ph.to_numpy()))
    print(f"[sort] absorption over {n} sorted axions ({per_cell}/cell): {runs[0][0]} photons",
          flush=True)
    for k, a, ph in runs[1:]:
        assert k == runs[0][0]
        for key in ("w", "id", "cell"):
            np.testing.assert_array_equal(a[key], runs[0][1][key])
            np.testing.assert_array_equal(ph[key], runs[0][2][key])
    assert runs[0][0] > 10
