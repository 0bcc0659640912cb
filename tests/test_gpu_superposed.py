"""Thermal emission by per-cell superposition on the GPU (needs an MI355X).

The oracle's superposed operator (oracle/axpic_oracle.c, pinned against the
per-electron law) runs on the same seeded plasma with its own cell weight
sums and its own per-cell channel coefficients, rounded to the precision the
kernels store them in (binary32 for fp32 plasmas), and must then draw the
same cell totals, pick the same electrons and sample the same energies:
counts, ids, cells and positions bit-exact, momenta and weights to 1e-6 (FP32
storage; energies from the quantile tables), exchange buffers to 1e-6.  Cases: lognormal weights with electrons
at the cap, no cap, fp32 and fp64, and the full-size 512x512 plasma, whose
integrated power must also match the closed form.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from oracle import analytic as A  # noqa: E402
from paper_2604_24627_amd import inputs as I  # noqa: E402
from paper_2604_24627_amd import axpic as B  # noqa: E402
from paper_2604_24627_amd.sim import AxpicSim  # noqa: E402

KEV_ERG = 1.602176634e-9


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def oracle_inputs(pl, o_cells, params, f32):
    """The oracle's view: the plasma's electrons in relative weights, and its own
    per-cell coefficients lambda_e / w_e = Gamma dt_phys w_ref_e / (w_a wa_mul) of
    eq. lambda_macro, stored in the kernels' precision."""
    e = pl["species"]["electrons"]
    osp = O.OSpecies(e["x"], e["p"], e["w"].astype(np.float64), e["id"], e["cell"])
    dtp = O.dt_phys(pl["grid"])
    coef = np.stack([o_cells["G_C"] * dtp * e["w_ref"] / (params["w_a"] * params["wa_mul"][1]),
                     o_cells["G_B"] * dtp * e["w_ref"] / (params["w_a"] * params["wa_mul"][2])])
    if f32:
        coef = coef.astype(np.float32).astype(np.float64)
    return osp, coef, e["off"]


def check_step(g, pl, o_cells, params, step):
    osp, coef, off = oracle_inputs(pl, o_cells, params, g.dtype == B.F32)
    n0, id0 = g.ax.n, g.next_id
    g.step_index = step
    g.fb.zero_()
    k = g.emit_thermal_cells()
    fb = np.zeros(g.ncell * 4)
    prod, Lam, N = O.emit_thermal_cells(g.grid_d, params, o_cells, osp, off, step, id0,
                                        fb=fb, coef_in=coef)
    assert k == prod["w"].size
    sl = slice(n0, n0 + k)
    np.testing.assert_array_equal(g.ax.id[sl].cpu().numpy().view(np.uint64), prod["id"])
    np.testing.assert_array_equal(g.ax.cell[sl].cpu().numpy(), prod["cell"])
    for d in range(g.ndim):
        np.testing.assert_array_equal(np64(g.ax.x[d][sl]), prod["x"][d])
    gp = np.stack([np64(g.ax.p[d][sl]) for d in range(3)])
    np.testing.assert_allclose(gp, prod["p"], rtol=1e-6, atol=1e-6 * np.abs(prod["p"]).max())
    np.testing.assert_allclose(np64(g.ax.w[sl]) * g.ax.w_ref, prod["w"], rtol=1e-6)
    torch.cuda.synchronize()
    np.testing.assert_allclose(g.fb.cpu().numpy(), fb, rtol=1e-6, atol=1e-9 * np.abs(fb).max())
    return k, Lam, N, prod


def test_cell_weight_sums():
    wl = I.Workload("w", ndim=2, n=(24, 20), ppc=37, dtype="f32", T_keV=3.0, n_e=6e25,
                    n_ref=6e25, lognormal_sigma=0.5, poisson_ppc=True, params=I.Params(channels=6))
    pl = I.make_plasma(wl, 1)
    print(f"[superposed] cell weights n={wl.n}", flush=True)
    g = AxpicSim(pl, wl.params, thermal="cells")
    e = pl["species"]["electrons"]
    off = e["off"]
    w = e["w"].astype(np.float64)
    W = np.array([w[off[c]:off[c + 1]].sum() for c in range(g.ncell)])
    M = np.array([w[off[c]:off[c + 1]].max() if off[c + 1] > off[c] else 0.0 for c in range(g.ncell)])
    cw = g.cellw.cpu().numpy()
    np.testing.assert_allclose(cw[: g.ncell], W, rtol=1e-14)
    np.testing.assert_array_equal(cw[g.ncell:], M)


@pytest.mark.parametrize("dtype,cap,n,ppc", [("f32", 0.25, (24, 20), 37),
                                             ("f32", float("inf"), (24, 20), 37),
                                             ("f64", 0.25, (24, 20), 37),
                                             ("f32", 0.25, (2, 2), 8000)])
def test_superposed_emission_matches_oracle(dtype, cap, n, ppc):
    """Three steps on both sides; with four cells of 8000 electrons a cell's products
    span several blocks of the events kernel."""
    p = I.Params(channels=6, g_ae=1e-13, w_a=2e-37, wa_mul=(1.0, 1.0, 0.08), lambda_cap=cap)
    wl = I.Workload("sup", ndim=2, n=n, ppc=ppc, dtype=dtype, T_keV=3.0, n_e=6e25,
                    n_ref=6e25, lognormal_sigma=0.5, params=p)
    pl = I.make_plasma(wl, 5)
    print(f"[superposed] workload n={wl.n} dtype={dtype} cap={cap}", flush=True)
    g = AxpicSim(pl, wl.params, thermal="cells")
    o = O.OracleSim(pl, wl.params, prec32=(dtype == "f32"))
    cells = o.cells()
    tot = 0
    for step in range(3):
        k, Lam, N, prod = check_step(g, pl, cells, o.params, step)
        tot += k
    assert tot > 3000
    if cap < 1.0 and ppc < 100:
        # electrons at the cap were picked (their products carry lambda_e / cap > 1; with
        # thousands per cell a macro-electron's weight, and mean, is too small for the cap)
        assert (np64(g.ax.w[: g.ax.n]) > np.array(wl.params.wa_mul)[1:].max() * 1.0000001).sum() > 50


def test_full_size_superposed_emission_matches_oracle_and_power():
    wl = I.config2()
    pl = I.make_plasma(wl, 0)
    print(f"[superposed] full-size plasma n={wl.n} ppc={wl.ppc}", flush=True)
    g = AxpicSim(pl, wl.params, thermal="cells")
    o = O.OracleSim(pl, wl.params, prec32=True)
    cells = o.cells()
    del o
    k, Lam, N, prod = check_step(g, pl, cells, I.config2().params.as_dict(), 0)
    print(f"[superposed] full-size thermal events {k}", flush=True)
    assert k > 20000
    del prod
    g.hist.zero_()
    g.step_index = 1
    for _ in range(6):
        g.step()
    h = g.hist_np()
    V = wl.ncell * wl.V_cell_cm3
    dtp = wl.dt / wl.omega0
    c0 = O.cell_state(wl.grid(), wl.params, np.array([wl.T_keV]), np.array([wl.n_e]),
                      [np.array([wl.n_e])], [1.0], [1.0])[0]
    for i, Q in ((1, c0["Q_C"]), (2, c0["Q_B"])):
        Qmc = h[i].sum() * KEV_ERG / (V * 6 * dtp)
        print(f"[superposed] channel {i}: MC power / closed form {Qmc / Q:.5f}", flush=True)
        assert Qmc == pytest.approx(Q, rel=0.015), i


def test_superposed_emission_with_empty_and_sparse_cells():
    """Poisson(3) electrons per cell: empty cells, single-electron cells, lognormal weights."""
    p = I.Params(channels=6, g_ae=1e-13, w_a=1e-38, wa_mul=(1.0, 1.0, 0.08), lambda_cap=0.5)
    wl = I.Workload("sparse", ndim=2, n=(40, 30), ppc=3, dtype="f32", T_keV=3.0, n_e=6e25,
                    n_ref=6e25, lognormal_sigma=0.5, poisson_ppc=True, params=p)
    pl = I.make_plasma(wl, 9)
    off = pl["species"]["electrons"]["off"]
    counts = np.diff(off)
    assert (counts == 0).sum() > 20 and (counts == 1).sum() > 50
    print(f"[superposed] sparse cells n={wl.n} empty={(counts == 0).sum()}", flush=True)
    g = AxpicSim(pl, wl.params, thermal="cells")
    o = O.OracleSim(pl, wl.params, prec32=True)
    cells = o.cells()
    tot = 0
    for step in range(4):
        k, Lam, N, prod = check_step(g, pl, cells, o.params, step)
        assert np.all(N[:, counts == 0] == 0)
        tot += k
    assert tot > 500
