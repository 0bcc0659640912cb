"""Parity of the HIP operators with the FP64 oracle (needs an MI355X).

Inputs are the seeded synthetic plasmas of paper_2604_24627_amd.inputs, at
sizes the oracle finishes in seconds that still span several 1024-particle
tiles and a ragged tail.  Bars:
  * integer work (event counts, product ids, absorption decisions, cell
    indices, push in binary32) is bit-exact.  Where a decision depends on a
    mean, both sides are fed the same seeded means (inputs.means) through the
    rate-fed entry; that the fused kernels decide exactly as when fed their
    own materialised means is checked on the GPU alone, and those means are
    checked against the oracle's own to the rate tolerance below;
  * FP32 rates within 1e-5 relative of the FP64 oracle; FP64 paths 1e-11;
  * sampled energies within 1e-6 relative (quantile-table accuracy 2e-8
    plus binary32 storage);
  * FP64 reductions (histograms, exchange buffers, moments) within 1e-9
    relative (summation order only).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_2604_24627_amd import inputs as I  # noqa: E402
from paper_2604_24627_amd import axpic as B  # noqa: E402
from paper_2604_24627_amd.sim import AxpicSim  # noqa: E402

ME = 510.99895


def small_workload(dtype="f32", n=(24, 20), ppc=37, T=3.0, ne=6e25, **pkw):
    p = I.Params(**pkw)
    wl = I.Workload("par", ndim=len(n), n=tuple(n), ppc=ppc, dtype=dtype, T_keV=T, n_e=ne,
                    n_ref=6e25, params=p)
    return wl


def pair(wl, seed=0, **kw):
    pl = I.make_plasma(wl, seed)
    print(f"[parity] workload={wl.name} n={wl.n} ppc={wl.ppc} dtype={wl.dtype} seed={seed}",
          flush=True)
    g = AxpicSim(pl, wl.params, **kw)
    o = O.OracleSim(pl, wl.params, prec32=(wl.dtype == "f32"))
    return g, o, pl


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_cell_state_matches_oracle():
    for Z, A in ((1, 1.0), (2, 4.0)):
        wl = small_workload(channels=7, inverse=1, g_ae=1e-13, boost=1e30)
        wl.Z, wl.A = Z, A
        g, o, _ = pair(wl)
        torch.cuda.synchronize()
        st = g.state.cpu().numpy().reshape(-1, B.STATE_N)
        oc = o.cells()
        for k, f in enumerate(["T", "n_e", "n_e_dep", "nZ", "nZ2", "rho", "XH", "kappa2", "G_P0",
                               "G_C", "G_B", "Q_C", "Q_B", "meanE_C", "meanE_B"]):
            np.testing.assert_allclose(st[:, k], oc[f], rtol=1e-12, atol=0, err_msg=f)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_rates_match_oracle(dtype):
    wl = small_workload(dtype, channels=7, inverse=1, g_ae=1e-13, g_agg_GeV=1e-10, boost=1e33,
                        w_a=1e-36)
    g, o, pl = pair(wl)
    rtol = 1e-5 if dtype == "f32" else 1e-11
    cells = o.cells()
    lamP = np64(g.rates(g.ph, B.PRIMAKOFF))
    _, olamP, _ = O.emit_primakoff(o.grid, o.params, cells, o.ph.copy(), 0, 1 << 40)
    np.testing.assert_allclose(lamP, olamP, rtol=rtol)
    lamC = np64(g.rates(g.el, B.COMPTON)); lamB = np64(g.rates(g.el, B.BREMS))
    _, olamT, _ = O.emit_thermal(o.grid, o.params, cells, o.el, 0, 1 << 40)
    np.testing.assert_allclose(lamC, olamT[0], rtol=rtol)
    np.testing.assert_allclose(lamB, olamT[1], rtol=rtol)
    # axions: a seeded population given to both sides
    axd = I.make_axions(wl, pl, 8.0, seed=11)
    g.load_axions(axd)
    assert g.ax.n > 1000
    pab = np64(g.rates(g.ax, B.COMPTON | B.BREMS))
    lag = np64(g.rates(g.ax, B.PRIMAKOFF))
    _, opab, olag, _, _ = O.absorb(o.grid, o.params, cells, O.OSpecies.from_input(axd), 0, 1 << 40)
    big = opab > 1e-30
    np.testing.assert_allclose(pab[big], opab[big], rtol=rtol * 3)
    assert np.all(pab[~big] <= 1e-30)
    # the a->gamma mean is taken before absorption here; compare where nothing was absorbed
    prm_noabs = dict(o.params, channels=1)
    _, _, olag2, _, _ = O.absorb(o.grid, prm_noabs, cells, O.OSpecies.from_input(axd), 0, 1 << 40)
    np.testing.assert_allclose(lag, olag2, rtol=rtol)


def _compare_products(gsp, n0, prod, w_ref, rtol_w, exact_p=True, rtol_p=1e-6):
    n = prod["w"].size
    assert gsp.n - n0 == n
    sl = slice(n0, n0 + n)
    gid = gsp.id[sl].cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(gid, prod["id"])
    np.testing.assert_array_equal(gsp.cell[sl].cpu().numpy(), prod["cell"])
    for d in range(gsp.ndim):
        np.testing.assert_array_equal(np64(gsp.x[d][sl]), prod["x"][d])
    gp = np.stack([np64(gsp.p[d][sl]) for d in range(3)])
    if exact_p:
        np.testing.assert_array_equal(gp, prod["p"])
    else:
        np.testing.assert_allclose(gp, prod["p"], rtol=rtol_p, atol=rtol_p * np.abs(prod["p"]).max())
    np.testing.assert_allclose(np64(gsp.w[sl]) * w_ref, prod["w"], rtol=rtol_w)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_primakoff_emission_bit_exact_counts(dtype):
    """Rate-fed conversion: both sides draw from the same seeded means (some above the
    cap), three steps in a row on the depleted photons."""
    wl = small_workload(dtype, channels=1, g_agg_GeV=1e-10, w_a=2e-35, lambda_cap=0.7)
    g, o, _ = pair(wl)
    cells = o.cells()
    for step in range(3):
        lam = I.means(g.ph.n, seed=100 + step, dtype=dtype)
        n0, id0 = g.ax.n, g.next_id
        g.step_index = step; o.step_index = step
        k = g.emit_primakoff(lam_in=dev(lam))
        prod, olam, K = O.emit_primakoff(o.grid, o.params, cells, o.ph, step, id0,
                                         o.hist, o.stats, lam_in=lam.astype(np.float64))
        assert k == prod["w"].size and k > 200
        _compare_products(g.ax, n0, prod, g.ax.w_ref, rtol_w=1e-6 if dtype == "f32" else 1e-13)
        np.testing.assert_allclose(np64(g.ph.w[: g.ph.n]) * g.ph.w_ref, o.ph.w,
                                   rtol=1e-6 if dtype == "f32" else 1e-13)
    torch.cuda.synchronize()
    np.testing.assert_allclose(g.hist_np().ravel(), o.hist, rtol=1e-10, atol=0)
    st = g.stats_dict()
    for nme in ("events_P", "num_P", "en_P", "capped"):
        assert st[nme] == pytest.approx(o.stats[O.ST[nme]], rel=1e-10), nme
    assert st["capped"] > 0


@pytest.mark.parametrize("mode", [0, 1])
def test_light_parents_bit_exact(mode):
    """Photons and axions around the product weight (lognormal weights, w' = w_ref):
    light_mode 0 converts a light parent whole with probability lambda w'/w, 1 draws the
    Poisson count.  Seeded means on both sides: three steps of photon conversion on the
    depleting photons, then a->gamma on a seeded axion population; every decision, id and
    product as the oracle's."""
    wl = small_workload("f32", channels=1, inverse=1, g_agg_GeV=1e-10, lambda_cap=4.0,
                        light_mode=mode)
    wl.lognormal_sigma = 0.5
    wph = I.make_plasma(wl, 0)["species"]["photons"]["w_ref"]
    wl.params.w_a = wph
    wl.params.w_gamma_prod = wph
    g, o, pl = pair(wl)
    cells = o.cells()
    for step in range(3):
        lam = I.means(g.ph.n, seed=150 + step, lo=1e-3, hi=2.0)
        light = o.ph.w < wph
        n0, id0 = g.ax.n, g.next_id
        g.step_index = step
        k = g.emit_primakoff(lam_in=dev(lam))
        prod, _, K = O.emit_primakoff(o.grid, o.params, cells, o.ph, step, id0, None, o.stats,
                                      lam_in=lam.astype(np.float64))
        print(f"[parity] light photons {int(light.sum())}/{light.size}, events {k}", flush=True)
        assert k == prod["w"].size and k > 100 and light.sum() > 100
        assert (K[light] > 0).sum() > 20
        if mode == 0:
            assert K[light].max() == 1
        _compare_products(g.ax, n0, prod, g.ax.w_ref, rtol_w=1e-6)
        np.testing.assert_allclose(np64(g.ph.w[: g.ph.n]) * g.ph.w_ref, o.ph.w, rtol=1e-6)
    st = g.stats_dict()
    assert st["overdepleted"] == o.stats[O.ST["overdepleted"]] > 0
    axd = I.make_axions(wl, pl, 12.0, seed=19)
    g.load_axions(axd)
    n = g.ax.n
    lag = I.means(n, seed=160, lo=1e-3, hi=2.0)
    osp = O.OSpecies.from_input(axd)
    light = (osp.w > 0) & (osp.w < wph)
    ph_n0, id0 = g.ph.n, g.next_id
    g.step_index = 3
    k = g.absorb(n, lam_in=dev(lag))
    prod, _, _, K, _ = O.absorb(o.grid, o.params, cells, osp, 3, id0,
                                lam_in=lag.astype(np.float64))
    print(f"[parity] light axions {int(light.sum())}/{n}, a->gamma photons {k}", flush=True)
    assert k == prod["w"].size and k > 100 and (K[light] > 0).sum() > 20
    if mode == 0:
        assert K[light].max() == 1
    _compare_products(g.ph, ph_n0, prod, g.ph.w_ref, rtol_w=1e-6)
    gw = np64(g.ax.w[:n]) * g.ax.w_ref
    np.testing.assert_array_equal(gw == 0.0, osp.w == 0.0)
    np.testing.assert_allclose(gw, osp.w, rtol=2e-6, atol=0)


@pytest.mark.parametrize("dtype,n,ppc", [("f32", (24, 20), 37), ("f64", (24, 20), 37),
                                          ("f32", (2, 2), 6000)])
def test_thermal_emission_matches_oracle(dtype, n, ppc):
    """Rate-fed Compton + brems emission from the same seeded means on both sides; with
    four cells of 6000 electrons a cell's products span many blocks of the events kernel
    (the exchange sums are stitched across them)."""
    wl = small_workload(dtype, n=n, ppc=ppc, channels=6, g_ae=1e-13, w_a=4e-38, lambda_cap=0.5)
    wl.params.wa_mul = (1.0, 1.0, 0.35)
    g, o, _ = pair(wl)
    cells = o.cells()
    fb_o = np.zeros(g.ncell * 4)
    for step in range(2):
        lam = I.means(g.el.n, seed=200 + step, rows=2, dtype=dtype)
        n0, id0 = g.ax.n, g.next_id
        g.step_index = step
        g.fb.zero_()
        k = g.emit_thermal(lam_in=dev(lam.reshape(-1)))
        fb_o[:] = 0.0
        prod, _, K = O.emit_thermal(o.grid, o.params, cells, o.el, step, id0, fb_o,
                                    o.hist, o.stats, lam_in=lam.astype(np.float64))
        assert k == prod["w"].size and k > 1000
        assert (prod["chan"] == 1).sum() > 300 and (prod["chan"] == 2).sum() > 300
        _compare_products(g.ax, n0, prod, g.ax.w_ref, rtol_w=1e-6 if dtype == "f32" else 1e-13,
                          exact_p=False, rtol_p=1e-6)
        torch.cuda.synchronize()
        np.testing.assert_allclose(g.fb.cpu().numpy(), fb_o, rtol=1e-6,
                                   atol=1e-9 * np.abs(fb_o).max())
    Eg = g.hist_np().ravel()
    # a product energy within the table error of a bin edge may land in the neighbour bin
    assert np.abs(Eg - o.hist).sum() <= 1e-6 * o.hist.sum() + 4 * (Eg.max() / 50)
    assert Eg.sum() == pytest.approx(o.hist.sum(), rel=1e-6)


def test_fused_thermal_counts_equal_rate_fed_counts():
    """The fused kernel decides exactly as when it is fed its own materialised means."""
    wl = small_workload("f32", channels=6, g_ae=1e-13, w_a=4e-38, lambda_cap=0.5)
    g1, _, pl = pair(wl)
    g2 = AxpicSim(pl, wl.params)
    lam = torch.stack([g2.rates(g2.el, B.COMPTON), g2.rates(g2.el, B.BREMS)]).contiguous()
    k1 = g1.emit_thermal()
    k2 = g2.emit_thermal(lam_in=lam.reshape(-1))
    assert k1 == k2
    a, b = g1.ax.to_numpy(), g2.ax.to_numpy()
    for key in ("w", "id", "cell"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(a["p"], b["p"])


@pytest.mark.parametrize("absorb_mode", [0, 1])
def test_fused_primakoff_and_absorption_equal_rate_fed(absorb_mode):
    """The fused conversion and absorption kernels decide exactly as when they are fed
    their own materialised means (GPU alone; the means themselves are checked against
    the oracle in test_rates_match_oracle), in deletion and in weight-reduction mode
    (where the a->gamma mean of the start-of-step weight is scaled by 1 - P_abs)."""
    wl = small_workload("f32", channels=7, inverse=1, g_ae=1e-13, g_agg_GeV=1e-10, boost=4e33,
                        w_a=1e-36, lambda_cap=1.0, absorb_mode=absorb_mode)
    g1, _, pl = pair(wl)
    g2 = AxpicSim(pl, wl.params)
    lam = g2.rates(g2.ph, B.PRIMAKOFF).clone()
    k1 = g1.emit_primakoff()
    k2 = g2.emit_primakoff(lam_in=lam)
    assert k1 == k2 > 100
    axd = I.make_axions(wl, pl, 16.0, seed=14)
    for g in (g1, g2):
        g.load_axions(axd)
        g.step_index = 2
    pab = g2.rates(g2.ax, B.COMPTON | B.BREMS).clone()
    lag = g2.rates(g2.ax, B.PRIMAKOFF).clone()
    n = g1.ax.n
    k1 = g1.absorb(n)
    k2 = g2.absorb(n, pabs_in=pab, lam_in=lag)
    assert k1 == k2
    for a, b in ((g1.ax, g2.ax), (g1.ph, g2.ph)):
        x, y = a.to_numpy(), b.to_numpy()
        for key in ("w", "id", "cell"):
            np.testing.assert_array_equal(x[key], y[key])
        np.testing.assert_array_equal(x["p"], y["p"])
    if absorb_mode == 0:
        assert (g1.ax.to_numpy()["w"] == 0).sum() > (axd["w"] == 0).sum() + 20
    else:
        assert k1 > 20 and np.all(g1.ax.to_numpy()["w"] <= axd["w"])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_push_and_binning_bit_exact(dtype):
    wl = small_workload(dtype, channels=1, g_agg_GeV=1e-10, w_a=2e-35)
    g, o, pl = pair(wl)
    axd = I.make_axions(wl, pl, 8.0, seed=12)
    g.load_axions(axd)
    osp = O.OSpecies.from_input(axd)
    for _ in range(7):
        g.bin_axions(push=True)
        O.push(o.grid, osp, dtype == "f32")
    b = g.ax.to_numpy()
    for d in range(2):
        np.testing.assert_array_equal(b["x"][d].astype(np.float64), osp.x[d])
    np.testing.assert_array_equal(b["cell"], osp.cell)


@pytest.mark.parametrize("mode,sort,n,per_cell", [(0, False, (24, 20), 12.0),
                                                  (1, False, (24, 20), 12.0),
                                                  (0, True, (24, 20), 12.0),
                                                  (1, True, (3, 2), 2500.0)])
def test_absorption_decisions_bit_exact(mode, sort, n, per_cell):
    """Rate-fed absorption (delete or reduce) and a->gamma on a seeded axion population,
    both sides given the same seeded probabilities and means.  In cell order (sorted) the
    exchange is summed without atomics, also over cells spanning several blocks."""
    wl = small_workload("f32", n=n, channels=7, inverse=1, g_ae=1e-13, g_agg_GeV=1e-10,
                        boost=4e33, w_a=1e-36, lambda_cap=1.0, absorb_mode=mode)
    g, o, pl = pair(wl)
    cells = o.cells()
    axd = I.make_axions(wl, pl, per_cell, seed=13 + mode)
    g.load_axions(axd)
    osp = O.OSpecies.from_input(axd)
    if sort:
        g.sort_axions()
        osp.sort_cells(g.ncell)
        assert g.ax.off is not None and g.ax.n_sorted == g.ax.n
    n = g.ax.n
    assert n > 2000
    pab = I.means(n, seed=30, lo=1e-5, hi=0.6)
    lag = I.means(n, seed=31, lo=1e-4, hi=2.0)
    g.fb.zero_()
    ph_n0, id0 = g.ph.n, g.next_id
    g.step_index = 3
    st0 = g.stats_dict()
    k = g.absorb(n, pabs_in=dev(pab), lam_in=dev(lag))
    fb_o = np.zeros(g.ncell * 4)
    st_o = np.zeros(O.ST_COUNT)
    prm = dict(o.params, w_gamma_prod=g.ph.w_ref)
    prod, _, _, K, dead = O.absorb(o.grid, prm, cells, osp, 3, id0, fb_o, st_o,
                                   pabs_in=pab.astype(np.float64),
                                   lam_in=lag.astype(np.float64))
    assert k == prod["w"].size
    gw = np64(g.ax.w[:n]) * g.ax.w_ref
    np.testing.assert_array_equal(gw == 0.0, osp.w == 0.0)
    np.testing.assert_allclose(gw, osp.w, rtol=2e-6, atol=0)
    assert k > 100
    if mode == 0:
        assert dead.sum() > 50
    _compare_products(g.ph, ph_n0, prod, g.ph.w_ref, rtol_w=1e-6)
    torch.cuda.synchronize()
    np.testing.assert_allclose(g.fb.cpu().numpy(), fb_o, rtol=1e-6, atol=1e-9 * np.abs(fb_o).max())
    st = g.stats_dict()
    assert st["abs_num"] - st0["abs_num"] == pytest.approx(st_o[O.ST["abs_num"]], rel=1e-6)


@pytest.mark.parametrize("ppc", [37, 64])
@pytest.mark.parametrize("scale", [80, 2000])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_feedback_matches_oracle(dtype, scale, ppc):
    """Moments, remapped momenta and T against the oracle (8 lanes per cell below 48
    electrons per cell, 16 from there on); at the larger exchange many cells cannot give
    the energy asked of them (clamped, O10): their count and the energy left unapplied,
    summed in a fixed order, are the oracle's and repeat bit for bit."""
    wl = small_workload(dtype, ppc=ppc, channels=6, g_ae=1e-13, feedback=1, T_mode=2,
                        r_relax=0.3)
    g, o, pl = pair(wl)
    rng = np.random.default_rng(21)
    fb = rng.normal(0, 1, (g.ncell, 4)) * np.array([3e-3, 1e-3, 1e-3, 1e-3]) * scale
    g.fb.copy_(torch.from_numpy(fb.ravel()))
    mom = torch.zeros(g.ncell * 5, dtype=torch.float64, device="cuda")
    p_before = [g.el.p[d].clone() for d in range(3)]
    T_before = g.T.clone()
    g.stats.zero_()
    g.feedback(moments=mom)
    mo = np.zeros(g.ncell * 5)
    st = np.zeros(O.ST_COUNT)
    O.feedback(o.grid, o.params, pl["species"]["electrons"]["off"], o.el, fb.ravel(), o.T, st, mo)
    torch.cuda.synchronize()
    np.testing.assert_allclose(mom.cpu().numpy(), mo, rtol=1e-10, atol=1e-14 * np.abs(mo).max())
    gp = np.stack([np64(g.el.p[d][: g.el.n]) for d in range(3)])
    tol = 2e-6 if dtype == "f32" else 1e-11
    np.testing.assert_allclose(gp, o.el.p, rtol=tol, atol=tol * np.abs(o.el.p).max())
    np.testing.assert_allclose(g.T.cpu().numpy(), o.T, rtol=1e-10)
    gst = g.stats_dict()
    assert st[O.ST["clamped_cells"]] == gst["clamped_cells"]
    assert st[O.ST["cold_cells"]] == gst["cold_cells"]
    assert gst["unapplied_E"] == pytest.approx(st[O.ST["unapplied_E"]], rel=1e-9, abs=0)
    if scale > 100:
        assert gst["clamped_cells"] > 50
        # the same call again from the same state: the statistics repeat bit for bit
        first = g.stats.clone()
        for d in range(3):
            g.el.p[d].copy_(p_before[d])
        g.T.copy_(T_before)
        g.stats.zero_()
        g.feedback()
        torch.cuda.synchronize()
        assert torch.equal(g.stats, first)


def test_compaction_is_stable_and_exact():
    wl = small_workload("f32", channels=7, inverse=1, g_ae=1e-13, boost=4e33, w_a=1e-36,
                        lambda_cap=1.0)
    g, _, _ = pair(wl)
    for _ in range(4):
        g.step()
    before = g.ax.to_numpy()
    g.compact_axions()
    after = g.ax.to_numpy()
    keep = before["w"] > 0
    assert 0 < keep.sum() < keep.size
    for key in ("w", "id", "cell"):
        np.testing.assert_array_equal(after[key], before[key][keep])
    np.testing.assert_array_equal(after["p"], before["p"][:, keep])
    np.testing.assert_array_equal(after["x"][:2], before["x"][:2, keep])


def test_photon_p2_cache_changes_nothing():
    """The photons' |p|^2 kept beside p (read by the conversion count instead of p)
    gives the same steps, bit for bit, as p itself, through a->gamma appends and
    photon compaction; and the cache then equals |p|^2 of every photon."""
    wl = small_workload("f32", channels=7, inverse=1, g_ae=1e-13, boost=4e33, w_a=1e-36,
                        lambda_cap=1.0)
    pl = I.make_plasma(wl, 9)
    g = AxpicSim(pl, wl.params, compact_every=2)
    h = AxpicSim(pl, wl.params, compact_every=2)
    h.ph.with_p2, h.ph.p2, h.ph._S = False, None, None
    n0 = g.ph.n
    for _ in range(5):
        g.step()
        h.step()
    torch.cuda.synchronize()
    assert h.ph.p2 is None and g.ph.p2 is not None
    assert g.ph.n != n0 and g._spare.get(B.PHOTON) is not None
    for key in ("w", "id", "cell", "p", "x"):
        np.testing.assert_array_equal(g.ph.to_numpy()[key], h.ph.to_numpy()[key])
        np.testing.assert_array_equal(g.ax.to_numpy()[key], h.ax.to_numpy()[key])
    n = g.ph.n
    kept = g.ph.p2[:n].clone()
    g.ph.fill_p2(g.lib, g.sh)
    torch.cuda.synchronize()
    assert torch.equal(kept, g.ph.p2[:n])
    p = [g.ph.p[d][:n].double() for d in range(3)]
    np.testing.assert_allclose(np64(kept), np64(p[0] ** 2 + p[1] ** 2 + p[2] ** 2), rtol=1e-6)


def test_config1_full_run_matches_oracle():
    """Config 1 (1D, 64 cells, fp64, Primakoff, 100 steps): GPU and oracle run
    independently with fused rates; every axion and the histogram agree."""
    wl = I.config1()
    g, o, _ = pair(wl)
    for s in range(wl.steps):
        g.step()
        o.step()
    assert g.ax.n == o.ax.n and g.ax.n > 100000
    a = g.ax.to_numpy()
    np.testing.assert_array_equal(a["id"], o.ax.id)
    np.testing.assert_array_equal(a["cell"], o.ax.cell)
    np.testing.assert_allclose(a["x"][0], o.ax.x[0], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(a["p"], o.ax.p)
    np.testing.assert_allclose(a["w"] * g.ax.w_ref, o.ax.w, rtol=1e-13)
    np.testing.assert_allclose(g.hist_np().ravel(), o.hist, rtol=1e-10)
    d = g.diag()
    t = o.totals()
    assert d["N_a"] == pytest.approx(t["N_a"], rel=1e-12)
    assert d["U_a"] == pytest.approx(t["U_a"], rel=1e-12)


def test_capacity_overflow_rerun_is_bit_identical():
    wl = small_workload("f32", channels=7, g_ae=1e-13, g_agg_GeV=1e-10, w_a=1e-36, lambda_cap=1.0)
    pl = I.make_plasma(wl, 3)
    g1 = AxpicSim(pl, wl.params, axion_capacity=16)         # forces repeated growth
    g2 = AxpicSim(pl, wl.params, axion_capacity=10 ** 7)
    for _ in range(3):
        g1.step(); g2.step()
    a, b = g1.ax.to_numpy(), g2.ax.to_numpy()
    assert a["w"].size == b["w"].size > 1000
    for key in ("w", "id", "cell"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(a["p"], b["p"])
    # FP64 histogram bins are accumulated with atomics: equal up to summation order
    np.testing.assert_allclose(g1.hist_np(), g2.hist_np(), rtol=1e-12, atol=0)


@pytest.mark.parametrize("thermal,absorb_mode", [("particle", 0), ("cells", 1)])
def test_determinism_two_runs_bitwise(thermal, absorb_mode):
    """Two runs of the same steps (all channels forward and inverse, feedback, T evolved)
    agree bit for bit: the FP64 sums -- the exchange fb, the histograms, the statistics --
    take no floating-point atomics, so the remapped momenta and temperatures, and with
    them every later decision, are reproducible."""
    wl = small_workload("f32", channels=7, inverse=1, g_ae=1e-13, boost=4e33, w_a=1e-36,
                        lambda_cap=1.0, feedback=1, T_mode=2, absorb_mode=absorb_mode)
    pl = I.make_plasma(wl, 5)
    runs = []
    for _ in range(2):
        g = AxpicSim(pl, wl.params, thermal=thermal)
        for _ in range(5):
            g.step()
        torch.cuda.synchronize()
        runs.append((g.ax.to_numpy(), g.el.to_numpy(), g.T.cpu().numpy(), g.hist_np(),
                     g.fb.cpu().numpy(), g.stats.cpu().numpy()))
    (a1, e1, T1, h1, f1, s1), (a2, e2, T2, h2, f2, s2) = runs
    for key in ("w", "id", "cell", "p", "x"):
        np.testing.assert_array_equal(a1[key], a2[key])
    np.testing.assert_array_equal(e1["p"], e2["p"])
    np.testing.assert_array_equal(T1, T2)
    np.testing.assert_array_equal(h1, h2)
    np.testing.assert_array_equal(f1, f2)
    np.testing.assert_array_equal(s1, s2)
    assert np.count_nonzero(f1) > 10 and h1.sum() > 0 and a1["w"].size > 100


def test_empty_inputs_append_nothing():
    """Empty parent or axion buffers: the calls only write the status words."""
    wl = small_workload("f32", channels=7, inverse=1, g_ae=1e-13, w_a=1e-36)
    g, _, _ = pair(wl)
    g.status.fill_(-7)
    saved_n = g.ph.n
    g.ph.n = 0
    try:
        assert g.emit_primakoff() == 0
    finally:
        g.ph.n = saved_n
    st = g.status.cpu().numpy()
    assert st[0] == g.ax.n and st[1] == 0 and st[2] == 0
    assert g.absorb(0) == 0
    g.compact_axions()
    assert g.ax.n == 0


def test_chained_step_recovers_from_overflow_bit_identical():
    """A step issued as a device chain: with buffers far too small (no growth ahead) the
    overflowing call and everything after it are skipped, the buffer is grown and the
    calls repeated; the run must equal one with ample buffers."""
    wl = small_workload("f32", channels=7, inverse=1, g_ae=1e-13, g_agg_GeV=1e-10, boost=4e33,
                        w_a=1e-36, lambda_cap=1.0, feedback=1, T_mode=2)
    pl = I.make_plasma(wl, 0)
    print("[parity] chained step overflow", flush=True)
    big = AxpicSim(pl, wl.params, axion_capacity=400000, photon_extra=100000)
    small = AxpicSim(pl, wl.params, axion_capacity=64)
    small.grow_ahead = False
    for _ in range(4):
        big.step()
        small.step()
    # the small run overflowed and grew; the big one never had to
    assert small.ax.capacity > 64 and big.ax.capacity == 400000
    assert small.ax.n == big.ax.n > 2000
    assert small.next_id == big.next_id
    for a, b in ((small.ax, big.ax), (small.ph, big.ph)):
        x, y = a.to_numpy(), b.to_numpy()
        for k in ("w", "id", "cell"):
            np.testing.assert_array_equal(x[k], y[k])
        np.testing.assert_array_equal(x["p"], y["p"])
    # the feedback's FP64 exchange sums are order-dependent at the 1e-16 level
    np.testing.assert_allclose(np64(small.el.p[0][: small.el.n]), np64(big.el.p[0][: big.el.n]),
                               rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(small.T.cpu().numpy(), big.T.cpu().numpy(), rtol=1e-7)
    np.testing.assert_allclose(small.hist_np(), big.hist_np(), rtol=1e-12)


def _nudge(x, k):
    """float32 array x moved by k[i] units in the last place (towards +inf for k > 0)."""
    x = np.asarray(x, dtype=np.float32).copy()
    for s in range(1, int(np.abs(k).max()) + 1):
        up, dn = k >= s, k <= -s
        x[up] = np.nextafter(x[up], np.float32(np.inf))
        x[dn] = np.nextafter(x[dn], np.float32(-np.inf))
    return x


def _uniforms(seed, ids, step, stream):
    """The oracle's two uniforms u53(r0, r1), u53(r2, r3) of each parent's draw, and the
    leading 24-bit bounds of the first word of each pair."""
    r = np.array([O.draw(seed, int(i), step, stream, 0) for i in ids], dtype=np.uint64)
    u = [np.array([O.u53(a, b) for a, b in r[:, q:q + 2]]) for q in (0, 2)]
    hi = [((r[:, q] >> 8) + 1).astype(np.float64) * 2.0 ** -24 for q in (0, 2)]
    lo = [(r[:, q] >> 8).astype(np.float64) * 2.0 ** -24 for q in (0, 2)]
    return u, lo, hi


def _boundary_means(u, hi, seed):
    """Means placed on the decisions of the Poisson inversion for uniform u: the 0/1
    boundary exp(-lam) = u, the FP64 shortcut 1 - lam = u, the FP32 pre-test bound
    1 - lam - 2^-22 = u_hi, and seeded means; each moved by -3 .. 3 ulps."""
    n = u.size
    j = np.arange(n)
    kind, k = j % 4, (j // 4) % 7 - 3
    base = np.where(kind == 0, -np.log(u), np.where(kind == 1, 1.0 - u, 1.0 - hi - 2.0 ** -22))
    base = np.where(base > 1e-30, base, 1e-7)
    lam = _nudge(base.astype(np.float32), k)
    lam[kind == 3] = I.means(n, seed=seed)[kind == 3]
    return np.maximum(lam, np.float32(1e-30)), kind


def test_count_pretests_at_decision_boundaries():
    """The count kernels decide surely-zero draws with FP32 tests on the leading 24 bits
    of the uniform before the FP64 inversion.  Means placed within a few ulps of every
    decision boundary (Poisson 0/1, the FP64 shortcut, the FP32 bound, Bernoulli
    absorption u < P, light-parent conversion u < lam w'/w) and parent weights within
    ulps of the light/heavy threshold: every count, id and product as the oracle's."""
    wl = small_workload("f32", channels=7, inverse=1, g_ae=1e-13, g_agg_GeV=1e-10,
                        boost=4e33, lambda_cap=64.0, light_mode=0)
    wph = I.make_plasma(wl, 0)["species"]["photons"]["w_ref"]
    wl.params.w_a = wph / 400.0                 # Primakoff products weigh w_a * 400 = w_ph
    wl.params.wa_mul = (400.0, 1.0, 1.0)
    wl.params.w_gamma_prod = wph
    g, o, pl = pair(wl)
    cells = o.cells()
    seed = int(wl.params.seed)
    # photons: a third lighter, a third heavier, a third within ulps of one product
    n = g.ph.n
    j = np.arange(n)
    w = np.where(j % 3 == 0, 0.5, np.where(j % 3 == 1, 2.0, 1.0)).astype(np.float32)
    w[j % 3 == 2] = _nudge(w[j % 3 == 2], (j[j % 3 == 2] // 3) % 5 - 2)
    g.ph.w[:n].copy_(dev(w))
    o.ph.w = w.astype(np.float64) * g.ph.w_ref
    (u, _), _, (hi, _) = _uniforms(seed, o.ph.id, 0, 0)
    lam, kind = _boundary_means(u, hi, seed=201)
    n0, id0 = g.ax.n, g.next_id
    g.step_index = 0
    k = g.emit_primakoff(lam_in=dev(lam))
    prod, _, K = O.emit_primakoff(o.grid, o.params, cells, o.ph, 0, id0, None, o.stats,
                                  lam_in=lam.astype(np.float64))
    print(f"[parity] boundary photons: {k} events, K>0 on the exp boundary "
          f"{int((K[kind == 0] > 0).sum())}/{int((kind == 0).sum())}", flush=True)
    assert k == prod["w"].size
    assert 0 < (K[kind == 0] > 0).sum() < (kind == 0).sum()
    _compare_products(g.ax, n0, prod, g.ax.w_ref, rtol_w=1e-6)
    np.testing.assert_allclose(np64(g.ph.w[:n]) * g.ph.w_ref, o.ph.w, rtol=1e-6)
    # electrons: both channels on their boundaries
    ne = g.el.n
    (uC, uB), _, (hC, hB) = _uniforms(seed, o.el.id, 0, 1)
    lC, _ = _boundary_means(uC, hC, seed=202)
    lB, _ = _boundary_means(uB[::-1].copy(), hB[::-1].copy(), seed=203)
    lB = lB[::-1].copy()
    lamT = np.concatenate([lC, lB])
    n0, id0 = g.ax.n, g.next_id
    k = g.emit_thermal(lam_in=dev(lamT))
    prodT, _, KT = O.emit_thermal(o.grid, o.params, cells, o.el, 0, id0,
                                  lam_in=lamT.reshape(2, ne).astype(np.float64))
    assert k == prodT["w"].size and k > 1000
    _compare_products(g.ax, n0, prodT, g.ax.w_ref, rtol_w=1e-6, exact_p=False)
    # axions: absorption probabilities on u, a->gamma means on both conversion rules
    axd = I.make_axions(wl, pl, 12.0, seed=23)
    # relative weights (w_ref = w_ph / 400): light ones as drawn, a fifth at 800 (heavier
    # than one photon product), a fifth within ulps of 400 (one product)
    ja = np.arange(axd["w"].size)
    wa = axd["w"].astype(np.float32)
    live = wa > 0
    wa[live & (ja % 5 == 1)] = 800.0
    thr = live & (ja % 5 == 2)
    wa[thr] = _nudge(np.full(int(thr.sum()), 400.0, np.float32), (ja[thr] // 5) % 5 - 2)
    axd["w"] = wa
    g.load_axions(axd)
    na = g.ax.n
    osp = O.OSpecies.from_input(axd)
    (ua, ug), (la, _), (ha, hg) = _uniforms(seed, osp.id, 3, 4)
    ja = np.arange(na)
    ka = (ja // 3) % 7 - 3
    pab = _nudge(np.where(ja % 3 == 0, ua, np.where(ja % 3 == 1, la, ha)).astype(np.float32), ka)
    pab = np.clip(pab, 0.0, 1.0).astype(np.float32)
    light = (osp.w > 0) & (osp.w < wph)
    heavy = (osp.w > 0) & ~light
    # a light axion converts iff u < lam w'/w: means with lam w'/w on u
    conv_lam = np.where(light, ug * osp.w / wph, 0.0)
    lag, _ = _boundary_means(ug, hg, seed=204)
    lag = np.where(light & (ja % 2 == 0), _nudge(conv_lam.astype(np.float32), ka), lag)
    lag = np.maximum(lag, np.float32(1e-30)).astype(np.float32)
    g.step_index = 3
    ph_n0, id0 = g.ph.n, g.next_id
    k = g.absorb(na, pabs_in=dev(pab), lam_in=dev(lag))
    prm = dict(o.params, w_gamma_prod=g.ph.w_ref)
    prodA, _, _, KA, dead = O.absorb(o.grid, prm, cells, osp, 3, id0, pabs_in=pab.astype(np.float64),
                                     lam_in=lag.astype(np.float64))
    print(f"[parity] boundary axions: {int(dead.sum())} absorbed of {na}, {k} photons, "
          f"light {int(light.sum())}", flush=True)
    assert k == prodA["w"].size and dead.sum() > 100 and light.sum() > 100
    assert (KA[light] > 0).sum() > 20 and (KA[heavy] > 0).sum() > 20
    gw = np64(g.ax.w[:na]) * g.ax.w_ref
    np.testing.assert_array_equal(gw == 0.0, osp.w == 0.0)
    _compare_products(g.ph, ph_n0, prodA, g.ph.w_ref, rtol_w=1e-6)


@pytest.mark.parametrize("ppc,poisson", [(2, True), (6, True), (37, False)])
def test_primakoff_cells_from_offsets_equal_cell_index(ppc, poisson):
    """Tiles of the cell-ordered photons take their cells from the per-cell offsets and
    their cells' prefactors from LDS when they span at most 256 cells (Poisson counts
    leave empty cells); sparser tiles, the ragged tail and buffers without offsets read
    the per-photon cell index.  All three decide exactly as the rate-fed path."""
    wl = small_workload("f32", n=(64, 64), ppc=ppc, channels=1, g_agg_GeV=1e-10, w_a=2e-35,
                        lambda_cap=0.7)
    wl.poisson_ppc = poisson
    pl = I.make_plasma(wl, 5)
    off = pl["species"]["photons"]["off"]
    print(f"[parity] ppc={ppc} poisson={poisson}: {int(off[-1])} photons, "
          f"{int((np.diff(off) == 0).sum())} empty cells", flush=True)
    g1 = AxpicSim(pl, wl.params)
    g2 = AxpicSim(pl, wl.params)
    g2.ph.off, g2.ph.n_sorted = None, 0
    g3 = AxpicSim(pl, wl.params)
    lam = g3.rates(g3.ph, B.PRIMAKOFF).clone()
    k1, k2, k3 = g1.emit_primakoff(), g2.emit_primakoff(), g3.emit_primakoff(lam_in=lam)
    assert k1 == k2 == k3 > 20
    for ga in (g2, g3):
        for a, b in ((g1.ax, ga.ax), (g1.ph, ga.ph)):
            x, y = a.to_numpy(), b.to_numpy()
            for key in ("w", "id", "cell"):
                np.testing.assert_array_equal(x[key], y[key])
            np.testing.assert_array_equal(x["p"], y["p"])


def test_cells_outside_the_domain_are_flagged_and_inert():
    """A cell whose temperature is NaN or negative, or whose electron density is negative,
    is flagged in its state record and gets zero prefactors (no event can happen there);
    every other cell keeps its prefactors bit for bit."""
    wl = small_workload("f32", channels=7, inverse=1, g_ae=1e-13)
    g, _, _ = pair(wl)
    before = g.pref64.clone().view(-1, B.PREF_N)
    assert g.domain_cells() == 0
    bad = [3, 5, 7]
    g.T[3] = float("nan")
    g.T[5] = -1.0
    g.dens[7] = -2.0
    g.cell_state()
    torch.cuda.synchronize()
    after = g.pref64.view(-1, B.PREF_N)
    assert g.domain_cells() == 3
    assert torch.all(after[bad] == 0.0)
    assert torch.all(g.pref32.view(-1, B.PREF_N)[bad] == 0.0)
    keep = torch.ones(g.ncell, dtype=torch.bool, device=after.device)
    keep[bad] = False
    assert torch.equal(after[keep], before[keep])
    flags = g.state.view(-1, B.STATE_N)[:, B.STATE_N - 1]
    assert torch.equal(torch.nonzero(flags).flatten().cpu(), torch.tensor(bad))
