"""The workloads at their own shapes (needs an MI355X).

* The all-channel forward plasma at full size (2D 512x512, 64 per cell per
  species, fp32), which is the launch configuration of the benchmark.  The
  means the fused count kernels compute, materialised, must agree with the
  oracle's own to 1e-5 for every photon and electron; the fused kernels must
  decide exactly as the rate-fed path fed those means (GPU alone); and with
  the same seeded means fed to both sides, every one of the 16.8M photons'
  and 16.8M electrons' event counts, product ids, cells and momenta must
  equal the oracle's.  The integrated power of the channels over a few
  steps must match the closed-form emissivities.
* The graded 3D plasma with Poisson per-cell counts, in the large-plasma
  recipe at a size the oracle runs whole: the same three checks for one
  step, then the feedback and temperature update element by element.
* Forward + inverse relaxation with lognormal weights and a macro-weight
  ratio of 100, one thermal channel at a time.  The axion number per energy
  bin must follow the detailed-balance recursion, which has a closed form.
  The Primakoff pair must conserve number and energy.  With feedback on, the
  plasma's kinetic energy plus the axions' energy must be constant (FP64).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from oracle import analytic as A  # noqa: E402
from paper_2604_24627_amd import inputs as I  # noqa: E402
from paper_2604_24627_amd import axpic as B  # noqa: E402
from paper_2604_24627_amd.sim import AxpicSim  # noqa: E402

ME = 510.99895
HBARC = 1.973269804e-8          # keV cm
KEV_ERG = 1.602176634e-9


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def same_population(a, b):
    x, y = a.to_numpy(), b.to_numpy()
    assert a.n == b.n
    for key in ("w", "id", "cell"):
        np.testing.assert_array_equal(x[key], y[key])
    np.testing.assert_array_equal(x["p"], y["p"])
    np.testing.assert_array_equal(x["x"], y["x"])


def check_means_and_fused(g, pl, wl, o, cells):
    """Materialised means against the oracle's own; then a second simulation fed
    those means must emit exactly what the fused kernels of `g` emit."""
    lamP = g.rates(g.ph, B.PRIMAKOFF).clone()
    lamT = torch.stack([g.rates(g.el, B.COMPTON), g.rates(g.el, B.BREMS)]).contiguous()
    _, olamP, _ = O.emit_primakoff(o.grid, o.params, cells, o.ph.copy(), 0, 1 << 40)
    np.testing.assert_allclose(np64(lamP), olamP, rtol=1e-5)
    del olamP
    _, olamT, _ = O.emit_thermal(o.grid, o.params, cells, o.el.copy(), 0, 1 << 40)
    np.testing.assert_allclose(np64(lamT), olamT, rtol=1e-5)
    del olamT
    g2 = AxpicSim(pl, wl.params)
    g.fb.zero_(); g2.fb.zero_()
    kP, kP2 = g.emit_primakoff(), g2.emit_primakoff(lam_in=lamP)
    kT, kT2 = g.emit_thermal(), g2.emit_thermal(lam_in=lamT.reshape(-1))
    print(f"[configs] fused vs rate-fed: Primakoff {kP}/{kP2}, thermal {kT}/{kT2}", flush=True)
    assert kP == kP2 and kT == kT2 and kP > 200 and kT > 200
    same_population(g.ax, g2.ax)
    np.testing.assert_array_equal(np64(g.ph.w[: g.ph.n]), np64(g2.ph.w[: g2.ph.n]))
    torch.cuda.synchronize()
    np.testing.assert_allclose(g.fb.cpu().numpy(), g2.fb.cpu().numpy(), rtol=1e-12, atol=0)


def products_equal(gsp, n0, prod, w_ref, exact_p, rtol_w=1e-6, rtol_p=1e-6):
    n = prod["w"].size
    assert gsp.n - n0 == n
    sl = slice(n0, n0 + n)
    np.testing.assert_array_equal(gsp.id[sl].cpu().numpy().view(np.uint64), prod["id"])
    np.testing.assert_array_equal(gsp.cell[sl].cpu().numpy(), prod["cell"])
    for d in range(gsp.ndim):
        np.testing.assert_array_equal(np64(gsp.x[d][sl]), prod["x"][d])
    gp = np.stack([np64(gsp.p[d][sl]) for d in range(3)])
    if exact_p:
        np.testing.assert_array_equal(gp, prod["p"])
    else:
        np.testing.assert_allclose(gp, prod["p"], rtol=rtol_p, atol=rtol_p * np.abs(prod["p"]).max())
    np.testing.assert_allclose(np64(gsp.w[sl]) * w_ref, prod["w"], rtol=rtol_w)


def test_full_size_forward_plasma_bit_exact_and_power():
    wl = I.config2()
    pl = I.make_plasma(wl, 0)
    print(f"[configs] full-size forward plasma n={wl.n} ppc={wl.ppc} dtype={wl.dtype}", flush=True)
    g = AxpicSim(pl, wl.params)
    o = O.OracleSim(pl, wl.params, prec32=True)
    cells = o.cells()
    st = g.state.cpu().numpy().reshape(-1, B.STATE_N)
    for k, f in enumerate(["T", "n_e", "n_e_dep", "nZ", "nZ2", "rho", "XH", "kappa2", "G_P0",
                           "G_C", "G_B"]):
        np.testing.assert_allclose(st[:, k], cells[f], rtol=1e-12, atol=0, err_msg=f)
    # the fused kernels as the step runs them: their means against the oracle's own, their
    # decisions against the rate-fed path fed those means
    check_means_and_fused(g, pl, wl, o, cells)
    # the same seeded means on both sides: every decision, id, cell and momentum
    g3 = AxpicSim(pl, wl.params)
    del pl
    lamP = I.means(g3.ph.n, seed=41, lo=1e-5, hi=2.0)
    n0, id0 = g3.ax.n, g3.next_id
    kP = g3.emit_primakoff(lam_in=dev(lamP))
    prodP, _, _ = O.emit_primakoff(o.grid, o.params, cells, o.ph, 0, id0,
                                   lam_in=lamP.astype(np.float64))
    print(f"[configs] Primakoff events {kP}", flush=True)
    assert kP == prodP["w"].size and kP > 10000
    products_equal(g3.ax, n0, prodP, g3.ax.w_ref, exact_p=True)
    np.testing.assert_allclose(np64(g3.ph.w[: g3.ph.n]) * g3.ph.w_ref, o.ph.w, rtol=1e-6)
    del prodP, lamP
    lamT = I.means(g3.el.n, seed=42, rows=2, lo=1e-5, hi=0.5)
    n0, id0 = g3.ax.n, g3.next_id
    g3.fb.zero_()
    kT = g3.emit_thermal(lam_in=dev(lamT.reshape(-1)))
    fb = np.zeros(g3.ncell * 4)
    prodT, _, _ = O.emit_thermal(o.grid, o.params, cells, o.el, 0, id0, fb,
                                 lam_in=lamT.astype(np.float64))
    print(f"[configs] thermal events {kT}", flush=True)
    assert kT == prodT["w"].size and kT > 20000
    products_equal(g3.ax, n0, prodT, g3.ax.w_ref, exact_p=False)
    torch.cuda.synchronize()
    np.testing.assert_allclose(g3.fb.cpu().numpy(), fb, rtol=1e-6, atol=1e-9 * np.abs(fb).max())
    del g3, prodT, lamT
    # integrated power of every channel over a few more full steps (the emission above was
    # step 0)
    del o
    g.step_index = 1
    for _ in range(4):
        g.step()
    h = g.hist_np()
    V = wl.ncell * wl.V_cell_cm3
    dtp = wl.dt / wl.omega0
    c0 = O.cell_state(wl.grid(), wl.params, np.array([wl.T_keV]), np.array([wl.n_e]),
                      [np.array([wl.n_e])], [1.0], [1.0])[0]
    QP = A.integrate_Q(A.dQdE_primakoff, 1e-4, 400.0, c0, wl.params)
    for i, Q in enumerate((QP, c0["Q_C"], c0["Q_B"])):
        Qmc = h[i].sum() * KEV_ERG / (V * g.step_index * dtp)
        print(f"[configs] channel {i}: MC power / closed form {Qmc / Q:.5f}", flush=True)
        assert Qmc == pytest.approx(Q, rel=0.015), i


def test_graded_poisson_plasma_one_step_elementwise():
    wl = I.config5(n=(24, 12, 10))
    wl.params.wa_mul = (50.0, 0.2, 0.1)
    wl.params.boost = 1.0
    wl.params.w_a = 3e-35
    pl = I.make_plasma(wl, 2)
    print(f"[configs] graded 3D plasma n={wl.n} Poisson ppc={wl.ppc}", flush=True)
    g = AxpicSim(pl, wl.params)
    o = O.OracleSim(pl, wl.params, prec32=True)
    cells = o.cells()
    st = g.state.cpu().numpy().reshape(-1, B.STATE_N)
    for k, f in enumerate(["T", "n_e", "n_e_dep", "nZ", "nZ2", "rho", "XH", "kappa2", "G_P0",
                           "G_C", "G_B"]):
        np.testing.assert_allclose(st[:, k], cells[f], rtol=1e-12, atol=0, err_msg=f)
    check_means_and_fused(g, pl, wl, o, cells)
    g = AxpicSim(pl, wl.params)
    lamP = I.means(g.ph.n, seed=43, lo=1e-4, hi=2.0)
    lamT = I.means(g.el.n, seed=44, rows=2, lo=1e-4, hi=2.0)
    g.fb.zero_()
    id0 = g.next_id
    kP = g.emit_primakoff(lam_in=dev(lamP))
    kT = g.emit_thermal(lam_in=dev(lamT.reshape(-1)))
    fb = np.zeros(g.ncell * 4)
    prodP, _, _ = O.emit_primakoff(o.grid, o.params, cells, o.ph, 0, id0,
                                   lam_in=lamP.astype(np.float64))
    prodT, _, _ = O.emit_thermal(o.grid, o.params, cells, o.el, 0, id0 + kP, fb,
                                 lam_in=lamT.astype(np.float64))
    print(f"[configs] events Primakoff {kP} thermal {kT}", flush=True)
    assert kP == prodP["w"].size and kT == prodT["w"].size and kP > 200 and kT > 200
    products_equal(g.ax, 0, dict((k, np.concatenate([prodP[k], prodT[k]], axis=-1))
                                 for k in ("w", "id", "cell", "x", "p")),
                   g.ax.w_ref, exact_p=False)
    torch.cuda.synchronize()
    np.testing.assert_allclose(g.fb.cpu().numpy(), fb, rtol=1e-6, atol=1e-9 * np.abs(fb).max())
    # the feedback and the temperature update of the step
    g.feedback()
    O.feedback(o.grid, o.params, o.el_off, o.el, fb, o.T)
    torch.cuda.synchronize()
    gp = np.stack([np64(g.el.p[d][: g.el.n]) for d in range(3)])
    np.testing.assert_allclose(gp, o.el.p, rtol=2e-6, atol=2e-6 * np.abs(o.el.p).max())
    np.testing.assert_allclose(g.T.cpu().numpy(), o.T, rtol=1e-7)


def _relax_workload(chan, T, boost, seed):
    p = I.Params(g_agg_GeV=1e-10, g_ae=1e-13, channels=chan, inverse=1, lambda_cap=1.0,
                 boost=boost, seed=seed, hist_lo_keV=1.5, hist_hi_keV=22.0, hist_nbins=8,
                 hist_log=1)
    wl = I.Workload("relax", ndim=2, n=(16, 16), ppc=32, dtype="f32", T_keV=T, n_e=6e25,
                    lognormal_sigma=0.5, params=p)
    wl.params.w_a = (wl.n_e * wl.V_cell_cm3 / wl.ppc) / 100.0
    return wl


@pytest.mark.parametrize("chan", [B.COMPTON, B.BREMS])
def test_relaxation_follows_detailed_balance_recursion(chan):
    """Emission E = V dn_eq/dE Gamma_abs dt per step and absorption
    p = 1 - exp(-Gamma_abs dt) of the axions present before the step give
    N_n(E) = V dn_eq/dE Gamma dt (1 - e^{-n Gamma dt}) / (1 - e^{-Gamma dt}).  The bin
    contents, the recursion's and their residuals come from the library's FP64
    equilibrium check on the GPU; the recursion's bin contents are also checked against
    the oracle's over the same seeded cells."""
    T = 3.0
    wl = _relax_workload(chan, T, 2e34, 3)
    pl = I.make_plasma(wl, 3)
    print(f"[configs] relaxation channel {chan} n={wl.n}", flush=True)
    g = AxpicSim(pl, wl.params, compact_every=16)
    steps = 300
    for _ in range(steps):
        g.step()
    r = g.equilibrium(t_steps=steps)
    # the recursion's content over the seeded plasma's own cells (the lognormal weights
    # give each cell its own density), from the oracle on the same seeded input
    o = O.OracleSim(pl, wl.params, prec32=True)
    ref = O.equilibrium(o.grid, o.params, o.cells(), O.OSpecies.empty(), t_steps=steps)
    np.testing.assert_allclose(r["nfix"], ref["nfix"], rtol=1e-9)
    z = r["z"][:8]
    print(f"[configs] relaxation channel {chan}: got/expected "
          f"{np.round(r['num'][:8] / r['nfix'][:8], 4)}, z {np.round(z, 2)}", flush=True)
    assert np.all(r["num"][:8] > 0) and np.all(np.abs(z) < 5.0), z


def test_primakoff_pair_conserves_number_and_energy():
    wl = _relax_workload(B.PRIMAKOFF, 1.3, 3e31, 5)
    pl = I.make_plasma(wl, 5)
    wl.params.w_a = pl["species"]["photons"]["w_ref"] / 100.0
    wl.params.w_gamma_prod = wl.params.w_a
    print(f"[configs] Primakoff pair n={wl.n}", flush=True)
    g = AxpicSim(pl, wl.params, compact_every=8)

    def totals():
        out = np.zeros(2)
        for sp in (g.ph, g.ax):
            d = sp.to_numpy()
            w = d["w"].astype(np.float64) * sp.w_ref
            E = ME * np.sqrt((d["p"].astype(np.float64) ** 2).sum(axis=0))
            out += np.array([w.sum(), (w * E).sum()])
        return out
    t0 = totals()
    share = []
    for s in range(120):
        g.step()
        if s % 20 == 19:
            np.testing.assert_allclose(totals(), t0, rtol=2e-5)
            share.append(float(g.ax.w[: g.ax.n].double().sum()) * g.ax.w_ref / t0[0])
    print(f"[configs] Primakoff axion number share {np.round(share, 5)}", flush=True)
    assert g.stats_dict()["ag_events"] > 0
    assert share[-1] > share[0] > 0.0


def test_feedback_conserves_plasma_plus_axion_energy_fp64():
    wl = _relax_workload(B.COMPTON | B.BREMS, 3.0, 3e34, 7)
    wl.dtype = "f64"
    wl.params.feedback, wl.params.T_mode = 1, 2
    pl = I.make_plasma(wl, 7)
    print(f"[configs] feedback energy n={wl.n} dtype=f64", flush=True)
    g = AxpicSim(pl, wl.params, compact_every=8)

    def energy():
        p2 = sum(g.el.p[d][: g.el.n] ** 2 for d in range(3))
        Ee = 0.5 * float((g.el.w[: g.el.n] * p2).sum()) * g.el.w_ref
        pa = torch.sqrt(sum(g.ax.p[d][: g.ax.n] ** 2 for d in range(3)))
        Ea = float((g.ax.w[: g.ax.n] * pa).sum()) * g.ax.w_ref
        return Ee + Ea, Ea
    e0, _ = energy()
    for _ in range(40):
        g.step()
        e, ea = energy()
        assert e == pytest.approx(e0, rel=1e-12)
    st = g.stats_dict()
    print(f"[configs] axion energy share {ea / e0:.3e}", flush=True)
    assert ea > 1e-6 * e0
    assert st["clamped_cells"] == 0 and st["cold_cells"] == 0
