"""Finite-mass axions on the GPU against the oracle (needs an MI355X).

Same bars as the massless parity tests, with m_a = 2 keV in a 3 keV plasma:
the means (Primakoff with the massive screened kernel and threshold, the
thermal rates cut at the mass, absorption with the massive equilibrium
density, a->gamma) to 1e-5 against the oracle's own; with seeded means on both
sides every count, id and cell bit-exact and momenta to 1e-6 (the products'
rescaled momenta are stored in binary32); the fused kernels equal the
rate-fed path on their own means; the sub-luminal push bit-exact; the cut
spectra's energies from the extended quantile tables to 1e-6; a full step
with feedback conserving plasma kinetic plus axion total energy (FP64).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_2604_24627_amd import inputs as I  # noqa: E402
from paper_2604_24627_amd import axpic as B  # noqa: E402
from paper_2604_24627_amd.sim import AxpicSim  # noqa: E402

ME = 510.99895
M_A = 2.0


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def workload(dtype="f32", n=(24, 20), ppc=37, **pkw):
    p = I.Params(m_a_keV=M_A, **pkw)
    return I.Workload("mass", ndim=len(n), n=tuple(n), ppc=ppc, dtype=dtype, T_keV=3.0, n_e=6e25,
                      n_ref=6e25, params=p)


def pair(wl, seed=0):
    pl = I.make_plasma(wl, seed)
    print(f"[mass] workload n={wl.n} ppc={wl.ppc} dtype={wl.dtype} m_a={M_A} keV seed={seed}",
          flush=True)
    return AxpicSim(pl, wl.params), O.OracleSim(pl, wl.params, prec32=(wl.dtype == "f32")), pl


def products(gsp, n0, prod, w_ref, rtol_p=1e-6):
    n = prod["w"].size
    assert gsp.n - n0 == n
    sl = slice(n0, n0 + n)
    np.testing.assert_array_equal(gsp.id[sl].cpu().numpy().view(np.uint64), prod["id"])
    np.testing.assert_array_equal(gsp.cell[sl].cpu().numpy(), prod["cell"])
    for d in range(gsp.ndim):
        np.testing.assert_array_equal(np64(gsp.x[d][sl]), prod["x"][d])
    gp = np.stack([np64(gsp.p[d][sl]) for d in range(3)])
    np.testing.assert_allclose(gp, prod["p"], rtol=rtol_p, atol=rtol_p * np.abs(prod["p"]).max())
    np.testing.assert_allclose(np64(gsp.w[sl]) * w_ref, prod["w"], rtol=1e-6)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_massive_rates_match_oracle(dtype):
    wl = workload(dtype, channels=7, inverse=1, g_ae=1e-13, g_agg_GeV=1e-10, boost=1e33,
                  w_a=1e-36)
    g, o, pl = pair(wl)
    rtol = 1e-5 if dtype == "f32" else 1e-9
    cells = o.cells()
    lamP = np64(g.rates(g.ph, B.PRIMAKOFF))
    _, olamP, _ = O.emit_primakoff(o.grid, o.params, cells, o.ph.copy(), 0, 1 << 40)
    E = ME * np.sqrt((pl["species"]["photons"]["p"].astype(np.float64) ** 2).sum(axis=0))
    below = E <= M_A
    assert below.sum() > 100 and np.all(lamP[below] == 0.0) and np.all(olamP[below] == 0.0)
    np.testing.assert_allclose(lamP[~below], olamP[~below], rtol=rtol)
    lamC, lamB = np64(g.rates(g.el, B.COMPTON)), np64(g.rates(g.el, B.BREMS))
    _, olamT, _ = O.emit_thermal(o.grid, o.params, cells, o.el.copy(), 0, 1 << 40)
    np.testing.assert_allclose(lamC, olamT[0], rtol=rtol)
    np.testing.assert_allclose(lamB, olamT[1], rtol=rtol)
    axd = I.make_axions(wl, pl, 8.0, seed=11)
    g.load_axions(axd)
    pab = np64(g.rates(g.ax, B.COMPTON | B.BREMS))
    lag = np64(g.rates(g.ax, B.PRIMAKOFF))
    _, opab, _, _, _ = O.absorb(o.grid, o.params, cells, O.OSpecies.from_input(axd), 0, 1 << 40)
    big = opab > 1e-30
    np.testing.assert_allclose(pab[big], opab[big], rtol=3 * rtol)
    assert np.all(pab[~big] <= 1e-30)
    prm_noabs = dict(o.params, channels=1)
    _, _, olag, _, _ = O.absorb(o.grid, prm_noabs, cells, O.OSpecies.from_input(axd), 0, 1 << 40)
    np.testing.assert_allclose(lag, olag, rtol=rtol)
    assert (lag > 0).sum() > 100


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_massive_primakoff_and_thermal_emission_bit_exact_counts(dtype):
    wl = workload(dtype, channels=7, g_ae=1e-13, g_agg_GeV=1e-10, w_a=2e-37, lambda_cap=0.7)
    g, o, pl = pair(wl)
    cells = o.cells()
    lam = I.means(g.ph.n, seed=300, dtype=dtype)
    n0, id0 = g.ax.n, g.next_id
    k = g.emit_primakoff(lam_in=dev(lam))
    prod, _, _ = O.emit_primakoff(o.grid, o.params, cells, o.ph, 0, id0, o.hist, o.stats,
                                  lam_in=lam.astype(np.float64))
    assert k == prod["w"].size and k > 200
    products(g.ax, n0, prod, g.ax.w_ref)
    np.testing.assert_allclose(np64(g.ph.w[: g.ph.n]) * g.ph.w_ref, o.ph.w, rtol=1e-6)
    lamT = I.means(g.el.n, seed=301, rows=2, dtype=dtype)
    n0, id0 = g.ax.n, g.next_id
    g.fb.zero_()
    k = g.emit_thermal(lam_in=dev(lamT.reshape(-1)))
    fb = np.zeros(g.ncell * 4)
    prod, _, _ = O.emit_thermal(o.grid, o.params, cells, o.el, 0, id0, fb, o.hist, o.stats,
                                lam_in=lamT.astype(np.float64))
    assert k == prod["w"].size and k > 1000
    products(g.ax, n0, prod, g.ax.w_ref)
    Ea = ME * np.sqrt((prod["p"] ** 2).sum(axis=0) + (M_A / ME) ** 2)
    assert Ea.min() > M_A
    torch.cuda.synchronize()
    np.testing.assert_allclose(g.fb.cpu().numpy(), fb, rtol=1e-6, atol=1e-9 * np.abs(fb).max())
    h = g.hist_np().ravel()
    assert h.sum() == pytest.approx(o.hist.sum(), rel=1e-6)


def test_massive_absorption_decisions_bit_exact():
    wl = workload("f32", channels=7, inverse=1, g_ae=1e-13, g_agg_GeV=1e-10, boost=4e33,
                  w_a=1e-36, lambda_cap=1.0)
    g, o, pl = pair(wl)
    cells = o.cells()
    axd = I.make_axions(wl, pl, 12.0, seed=13)
    g.load_axions(axd)
    n = g.ax.n
    pab = I.means(n, seed=32, lo=1e-5, hi=0.6)
    lag = I.means(n, seed=33, lo=1e-4, hi=2.0)
    osp = O.OSpecies.from_input(axd)
    g.fb.zero_()
    ph_n0, id0 = g.ph.n, g.next_id
    g.step_index = 3
    k = g.absorb(n, pabs_in=dev(pab), lam_in=dev(lag))
    fb_o = np.zeros(g.ncell * 4)
    prm = dict(o.params, w_gamma_prod=g.ph.w_ref)
    prod, _, _, K, dead = O.absorb(o.grid, prm, cells, osp, 3, id0, fb_o, None,
                                   pabs_in=pab.astype(np.float64), lam_in=lag.astype(np.float64))
    assert k == prod["w"].size and k > 100 and dead.sum() > 50
    gw = np64(g.ax.w[:n]) * g.ax.w_ref
    np.testing.assert_array_equal(gw == 0.0, osp.w == 0.0)
    np.testing.assert_allclose(gw, osp.w, rtol=2e-6, atol=0)
    products(g.ph, ph_n0, prod, g.ph.w_ref)
    torch.cuda.synchronize()
    np.testing.assert_allclose(g.fb.cpu().numpy(), fb_o, rtol=1e-6, atol=1e-9 * np.abs(fb_o).max())


def test_massive_fused_kernels_equal_rate_fed():
    wl = workload("f32", channels=7, inverse=1, g_ae=1e-13, g_agg_GeV=1e-10, boost=4e33,
                  w_a=1e-36, lambda_cap=1.0)
    g1, _, pl = pair(wl)
    g2 = AxpicSim(pl, wl.params)
    lam = g2.rates(g2.ph, B.PRIMAKOFF).clone()
    lamT = torch.stack([g2.rates(g2.el, B.COMPTON), g2.rates(g2.el, B.BREMS)]).contiguous()
    assert g1.emit_primakoff() == g2.emit_primakoff(lam_in=lam) > 100
    assert g1.emit_thermal() == g2.emit_thermal(lam_in=lamT.reshape(-1))
    axd = I.make_axions(wl, pl, 16.0, seed=14)
    for g in (g1, g2):
        g.load_axions(axd)
        g.step_index = 2
    pab = g2.rates(g2.ax, B.COMPTON | B.BREMS).clone()
    lag = g2.rates(g2.ax, B.PRIMAKOFF).clone()
    n = g1.ax.n
    assert g1.absorb(n) == g2.absorb(n, pabs_in=pab, lam_in=lag)
    for a, b in ((g1.ax, g2.ax), (g1.ph, g2.ph)):
        x, y = a.to_numpy(), b.to_numpy()
        for key in ("w", "id", "cell"):
            np.testing.assert_array_equal(x[key], y[key])
        np.testing.assert_array_equal(x["p"], y["p"])
    assert (g1.ax.to_numpy()["w"] == 0).sum() > (axd["w"] == 0).sum() + 20


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_massive_push_bit_exact(dtype):
    wl = workload(dtype, channels=1)
    g, o, pl = pair(wl)
    axd = I.make_axions(wl, pl, 8.0, seed=12)
    axd["p"] = (axd["p"].astype(np.float64) * 0.3).astype(axd["p"].dtype)   # slow: |p| ~ m
    g.load_axions(axd)
    osp = O.OSpecies.from_input(axd)
    for _ in range(7):
        g.bin_axions(push=True)
        O.push(o.grid, osp, dtype == "f32", M_A)
    b = g.ax.to_numpy()
    for d in range(2):
        np.testing.assert_array_equal(b["x"][d].astype(np.float64), osp.x[d])
    np.testing.assert_array_equal(b["cell"], osp.cell)


def test_massive_superposed_emission_matches_oracle():
    p = I.Params(channels=6, g_ae=1e-13, w_a=2e-37, wa_mul=(1.0, 1.0, 0.08), lambda_cap=0.25,
                 m_a_keV=M_A)
    wl = I.Workload("sup", ndim=2, n=(24, 20), ppc=37, dtype="f32", T_keV=3.0, n_e=6e25,
                    n_ref=6e25, lognormal_sigma=0.5, params=p)
    pl = I.make_plasma(wl, 5)
    g = AxpicSim(pl, wl.params, thermal="cells")
    o = O.OracleSim(pl, wl.params, prec32=True)
    cells = o.cells()
    e = pl["species"]["electrons"]
    osp = O.OSpecies(e["x"], e["p"], e["w"].astype(np.float64), e["id"], e["cell"])
    dtp = O.dt_phys(pl["grid"])
    prm = o.params
    T = cells["T"]
    qC = np.array([O.compton_ccdf(M_A / t) for t in T])
    qB = np.array([O.gammainc_Q(prm["brems_k"], M_A / (prm["brems_theta"] * t)) for t in T])
    coef = np.stack([cells["G_C"] * dtp * e["w_ref"] / (prm["w_a"] * prm["wa_mul"][1]) * qC,
                     cells["G_B"] * dtp * e["w_ref"] / (prm["w_a"] * prm["wa_mul"][2]) * qB])
    coef = coef.astype(np.float32).astype(np.float64)
    n0, id0 = g.ax.n, g.next_id
    g.fb.zero_()
    k = g.emit_thermal_cells()
    fb = np.zeros(g.ncell * 4)
    prod, _, _ = O.emit_thermal_cells(g.grid_d, prm, cells, osp, e["off"], 0, id0, fb=fb,
                                      coef_in=coef)
    assert k == prod["w"].size and k > 1000
    products(g.ax, n0, prod, g.ax.w_ref)
    torch.cuda.synchronize()
    np.testing.assert_allclose(g.fb.cpu().numpy(), fb, rtol=1e-6, atol=1e-9 * np.abs(fb).max())


def test_massive_full_step_conserves_energy_fp64():
    p = I.Params(channels=7, inverse=1, g_ae=1e-13, g_agg_GeV=1e-10, boost=3e34, lambda_cap=1.0,
                 feedback=1, T_mode=2, m_a_keV=M_A)
    wl = I.Workload("relax", ndim=2, n=(16, 16), ppc=32, dtype="f64", T_keV=3.0, n_e=6e25,
                    lognormal_sigma=0.5, params=p)
    wl.params.w_a = (wl.n_e * wl.V_cell_cm3 / wl.ppc) / 100.0
    pl = I.make_plasma(wl, 7)
    g = AxpicSim(pl, wl.params, compact_every=8)
    mu2 = (M_A / ME) ** 2

    def energy():
        p2e = sum(g.el.p[d][: g.el.n] ** 2 for d in range(3))
        Ee = 0.5 * float((g.el.w[: g.el.n] * p2e).sum()) * g.el.w_ref
        Ea = float((g.ax.w[: g.ax.n] * torch.sqrt(sum(g.ax.p[d][: g.ax.n] ** 2 for d in range(3))
                                                   + mu2)).sum()) * g.ax.w_ref
        return Ee, Ea
    # Primakoff conversions exchange energy with the photons, not the plasma: count them
    def photons():
        return float((g.ph.w[: g.ph.n] * torch.sqrt(sum(g.ph.p[d][: g.ph.n] ** 2
                                                        for d in range(3)))).sum()) * g.ph.w_ref
    e0 = sum(energy()) + photons()
    for _ in range(30):
        g.step()
    Ee, Ea = energy()
    assert Ee + Ea + photons() == pytest.approx(e0, rel=1e-12)
    d = g.diag()
    assert d["U_a"] == pytest.approx(Ea * ME, rel=1e-12)
    assert Ea > 1e-6 * e0
