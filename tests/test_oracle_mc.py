"""Statistical pins of the oracle's Monte-Carlo operators.

Each test runs the oracle's operators and compares with an expectation fixed
by the paper's construction: the unbiased macro-event yield (Sec. II.D),
the expected per-bin relaxation towards the detailed-balance fixed point
(Sec. II.I), the exact invariants of the bidirectional Primakoff conversion
(Sec. II.F.1) and of the conservative feedback (Sec. II.J), and invariance
under the axion macro-weight (App. A).  Tolerances are a few standard errors.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
from oracle import analytic as A
from paper_2604_24627_amd import inputs as I

ME = 510.99895
HBARC = 1.973269804e-8
ZETA3 = 1.2020569031595942854


def small_plasma(T=3.0, ne=6e25, ncell=4, ppc=2048, dtype="f64", seed=0, **pkw):
    p = I.Params(**pkw)
    wl = I.Workload("t", ndim=1, n=(ncell,), ppc=ppc, dtype=dtype, T_keV=T, n_e=ne, params=p)
    return wl, I.make_plasma(wl, seed)


def test_thermal_emission_yield_is_unbiased():
    """E[sum of product weights * E] over one step = Q V dt for each thermal channel,
    with and without Poisson-mean capping."""
    for cap, wa in ((math.inf, 4e-38), (0.1, 1e-39)):
        wl, pl = small_plasma(channels=6, g_ae=1e-13, w_a=wa, lambda_cap=cap, boost=1.0)
        sim = O.OracleSim(pl, wl.params)
        cells = sim.cells()
        st = np.zeros(O.ST_COUNT)
        tot = {1: [], 2: []}
        for s in range(10):
            prod, lam, K = O.emit_thermal(sim.grid, sim.params, cells, sim.el, s, 10 ** 9, stats=st)
            E = ME * np.sqrt((prod["p"] ** 2).sum(axis=0))
            for ch in (1, 2):
                m = prod["chan"] == ch
                tot[ch].append((prod["w"][m] * E[m], lam[ch - 1]))
        V = O.V_cell(sim.grid) * wl.ncell
        dt = O.dt_phys(sim.grid)
        c = cells[0]
        for ch, Q in ((1, c["Q_C"]), (2, c["Q_B"])):
            est = np.mean([t[0].sum() for t in tot[ch]]) * 1.602176634e-9 / (V * dt)
            # relative standard error from the number of events and the spread of E
            nev = sum(t[0].size for t in tot[ch])
            assert nev > 2000
            rel = 5 * 1.3 / math.sqrt(nev)
            assert est == pytest.approx(Q, rel=rel), (ch, cap, est / Q)
        if cap < math.inf:
            assert st[O.ST["capped"]] > 0


def test_primakoff_yield_matches_conditional_expectation():
    """E[sum w_a' E] = sum_photons w_gamma P(omega) omega, and the photon weight lost equals
    the axion weight made (number conservation, Sec. II.F.1)."""
    wl, pl = small_plasma(T=1.3, channels=1, g_agg_GeV=1e-10, w_a=1e-38, boost=1e3)
    sim = O.OracleSim(pl, wl.params)
    cells = sim.cells()
    dt = O.dt_phys(sim.grid)
    om = ME * np.sqrt((sim.ph.p ** 2).sum(axis=0))
    G = np.array([O.gamma_prim(cells[c], sim.params, o) for c, o in zip(sim.ph.cell, om)])
    expect = (sim.ph.w * -np.expm1(-G * dt) * om).sum()
    got = []
    for s in range(5):
        ph = sim.ph.copy()
        w0 = ph.w.sum()
        prod, lam, K = O.emit_primakoff(sim.grid, sim.params, cells, ph, s, 10 ** 9)
        E = ME * np.sqrt((prod["p"] ** 2).sum(axis=0))
        got.append((prod["w"] * E).sum())
        assert w0 - ph.w.sum() == pytest.approx(prod["w"].sum(), rel=1e-9)
    nev = prod["w"].size
    assert nev > 500
    assert np.mean(got) == pytest.approx(expect, rel=5 * 1.5 / math.sqrt(5 * nev))


@pytest.mark.parametrize("mode", [0, 1])
def test_light_parents_convert_whole(mode):
    """Parents lighter than one product (Sec. II.F.1 depletes by the converted weight and
    leaves this case open).  light_mode 0: a light parent converts whole with probability
    P = lambda w'/w, so the mean converted weight is sum w P; light_mode 1 (the Poisson
    count, whole conversion on K >= 1): probability 1 - exp(-lambda), a mean transfer of
    sum w (1 - e^-lambda), short of sum w P by about the factor w / w'.  Both for photons
    (photon -> axion, w' = w_a wa_mul[0]) and axions (a -> gamma, w' = w_gamma_prod)."""
    wl, pl = small_plasma(T=3.0, ncell=4, ppc=4096, channels=1, inverse=1, g_agg_GeV=1e-10,
                          light_mode=mode)
    wph = pl["species"]["photons"]["w_ref"]
    wl.params.w_a = 4.0 * wph
    wl.params.w_gamma_prod = 20.0 * wl.params.w_a
    sim = O.OracleSim(pl, wl.params)
    cells = sim.cells()
    rng = np.random.default_rng([17, mode])
    steps = 6

    def check(parents, wprod, run):
        n = parents.w.size
        P = rng.uniform(0.05, 0.6, n)
        lam = P * parents.w / wprod
        assert np.all(parents.w < wprod)
        q = P if mode == 0 else -np.expm1(-lam)
        expect = (parents.w * q).sum()
        sd = math.sqrt((parents.w ** 2 * q * (1.0 - q)).sum())
        moved = []
        for s in range(steps):
            sp = parents.copy()
            prod, K = run(sp, s, lam)
            whole = K > 0
            if mode == 0:
                assert K.max() == 1
            # a converted light parent is gone, its products carry its weight
            assert np.all(sp.w[whole] == 0.0) and np.all(sp.w[~whole] == parents.w[~whole])
            assert prod["w"].sum() == pytest.approx(parents.w[whole].sum(), rel=1e-12)
            moved.append(parents.w[whole].sum())
        z = (np.mean(moved) - expect) / (sd / math.sqrt(steps))
        assert abs(z) < 5.0, z
        return np.mean(moved), (parents.w * P).sum()

    def run_p(sp, s, lam):
        prod, _, K = O.emit_primakoff(sim.grid, sim.params, cells, sp, s, 10 ** 9, lam_in=lam)
        return prod, K

    got, unbiased = check(sim.ph, wl.params.w_a * wl.params.wa_mul[0], run_p)
    axd = I.make_axions(wl, pl, 512.0, seed=3, zero_frac=0.0)
    ax = O.OSpecies.from_input(axd)

    def run_a(sp, s, lam):
        prod, _, _, K, _ = O.absorb(sim.grid, sim.params, cells, sp, s, 10 ** 9, lam_in=lam)
        return prod, K

    got_a, unbiased_a = check(ax, wl.params.w_gamma_prod, run_a)
    if mode == 0:
        assert got == pytest.approx(unbiased, rel=0.02) and got_a == pytest.approx(unbiased_a, rel=0.02)
    else:
        assert got < 0.5 * unbiased and got_a < 0.8 * unbiased_a


def _bin_number(ax, edges):
    E = ME * np.sqrt((ax.p ** 2).sum(axis=0))
    return np.histogram(E, bins=edges, weights=ax.w)[0], np.histogram(E, bins=edges,
                                                                     weights=ax.w ** 2)[0]


@pytest.mark.parametrize("chan,mb", [(2, 0), (4, 1)])
def test_relaxation_follows_detailed_balance_recursion(chan, mb):
    """Forward + inverse thermal operators in one cell: the expected axion number per
    energy bin after t steps is n_eq(E) * g/(1 - e^-g) * (1 - e^-g t), g = Gamma_abs dt,
    which tends to the equilibrium spectrum n_eq as g -> 0 (Sec. II.I)."""
    T, ne = 3.0, 6e25
    wl, pl = small_plasma(T=T, ne=ne, ncell=1, ppc=4096, channels=chan, inverse=1, g_ae=1e-13,
                          boost=2e34, w_a=5e-5, lambda_cap=1.0, eq_stats=mb)
    sim = O.OracleSim(pl, wl.params)
    steps = 160
    for _ in range(steps):
        sim.step()
    c = sim.cells()[0]
    dt = O.dt_phys(sim.grid)
    V = O.V_cell(sim.grid)
    edges = np.array([1.0, 2.0, 3.0, 4.5, 6.0, 8.0, 11.0, 15.0, 22.0])

    def dneq(E):
        occ = math.exp(-E / T) if mb else 1.0 / math.expm1(E / T)
        return E * E / (2 * math.pi ** 2 * HBARC ** 3) * occ

    def expected(E):
        g = O.gamma_abs(c, sim.params, E)[0] * dt
        return V * dneq(E) * g / -math.expm1(-g) * -math.expm1(-g * steps)

    exp_bins = np.array([integrate.quad(expected, edges[k], edges[k + 1], epsrel=1e-9)[0]
                         for k in range(edges.size - 1)])
    got, w2 = _bin_number(sim.ax, edges)
    # axions are born one step before being eligible for absorption: the oracle's
    # operators absorb the start-of-step population only (Jacobi order), as the recursion.
    z = (got - exp_bins) / np.sqrt(np.maximum(w2, 1e-300) * 3.0)
    assert np.all(np.abs(z) < 5.0), (got / exp_bins, z)
    # equilibrium number density of a massless boson: zeta3 T^3 / (pi^2 (hbar c)^3)
    if mb == 0:
        Neq = ZETA3 * T ** 3 / (math.pi ** 2 * HBARC ** 3) * V
        full = integrate.quad(lambda E: V * dneq(E), 1e-9, 200)[0]
        assert full == pytest.approx(Neq, rel=1e-8)


def test_primakoff_pair_conserves_number_energy_momentum():
    """Forward and inverse Primakoff conversion conserve sum w, sum w E and sum w p exactly
    (up to rounding) every step, and drive the axion share towards the two-state fixed point."""
    wl, pl = small_plasma(T=1.3, ncell=2, ppc=512, channels=1, inverse=1, g_agg_GeV=1e-10,
                          boost=3e31, w_a=2e-5, lambda_cap=4.0)
    ph_wref = pl["species"]["photons"]["w_ref"]
    wl.params.w_gamma_prod = 2e-5
    sim = O.OracleSim(pl, wl.params)
    assert sim.pdict["w_gamma_prod"] == 2e-5 and ph_wref > 1e-5

    def tot():
        out = []
        for sp in (sim.ph, sim.ax):
            E = ME * np.sqrt((sp.p ** 2).sum(axis=0))
            out.append(np.array([sp.w.sum(), (sp.w * E).sum(), *(sp.w * sp.p).sum(axis=1)]))
        return out
    t0 = sum(tot())
    shares = []
    for s in range(30):
        sim.step()
        t = tot()
        np.testing.assert_allclose(t[0] + t[1], t0, rtol=1e-11, atol=1e-14 * abs(t0[1]))
        shares.append(t[1][0] / (t[0][0] + t[1][0]))
    assert shares[-1] > shares[0] > 0.0
    assert sim.stats[O.ST["ag_events"]] > 0


def test_full_step_conserves_plasma_plus_axion_energy():
    """With feedback on, the electrons' kinetic energy plus the axions' energy is constant
    every step (thermal channels only; Sec. II.J)."""
    wl, pl = small_plasma(T=3.0, ncell=8, ppc=256, channels=6, inverse=1, g_ae=1e-13,
                          boost=3e34, w_a=2e-4, lambda_cap=1.0, feedback=1, T_mode=2)
    sim = O.OracleSim(pl, wl.params)

    def energy():
        Ee = 0.5 * (sim.el.w * (sim.el.p ** 2).sum(axis=0)).sum()
        Ea = (sim.ax.w * np.sqrt((sim.ax.p ** 2).sum(axis=0))).sum()
        return Ee + Ea, Ea
    e0, _ = energy()
    for s in range(25):
        sim.step()
        e, ea = energy()
        assert e == pytest.approx(e0, rel=1e-12)
    assert ea > 1e-6 * e0
    assert sim.stats[O.ST["clamped_cells"]] == 0 and sim.stats[O.ST["cold_cells"]] == 0
    assert np.all(sim.T != 3.0)


def test_spectrum_invariant_under_axion_macro_weight():
    """App. A: the reconstructed brems spectrum does not depend on w_a (per-bin power agrees
    with the analytic expectation within Monte-Carlo noise for w_a and 100 w_a)."""
    edges = np.array([0.5, 1.5, 3.0, 5.0, 8.0, 12.0, 20.0])
    res = {}
    for wa in (2e-39, 2e-37):
        wl, pl = small_plasma(T=1.3, ncell=4, ppc=4096, channels=4, g_ae=1e-13, w_a=wa,
                              boost=3e3, lambda_cap=math.inf)
        sim = O.OracleSim(pl, wl.params)
        cells = sim.cells()
        H = np.zeros(edges.size - 1); H2 = np.zeros_like(H)
        for s in range(4):
            prod, lam, K = O.emit_thermal(sim.grid, sim.params, cells, sim.el, s, 10 ** 9)
            E = ME * np.sqrt((prod["p"] ** 2).sum(axis=0))
            H += np.histogram(E, bins=edges, weights=prod["w"] * E)[0]
            H2 += np.histogram(E, bins=edges, weights=(prod["w"] * E) ** 2)[0]
        V = O.V_cell(sim.grid) * wl.ncell
        scale = 1.602176634e-9 / (V * 4 * O.dt_phys(sim.grid) * 3e3)
        res[wa] = (H * scale, np.sqrt(H2) * scale)
        ref = np.array([integrate.quad(
            lambda e: float(A.dQdE_brems(np.array([e]), cells[0], sim.params)[0]),
            edges[k], edges[k + 1])[0] for k in range(edges.size - 1)])
        z = (res[wa][0] - ref) / res[wa][1]
        assert np.all(np.abs(z) < 5.0), (wa, z)
    assert res[2e-39][1].mean() < res[2e-37][1].mean()


def test_superposed_thermal_emission_has_the_per_electron_law():
    """Per-cell superposition: over many independent steps each electron's event count
    has mean min(lambda_e, cap) (chi-square over the electrons), the product weights
    carry lambda_e / cap for capped electrons so that the physical yield per electron
    is lambda_e w_prod, and a cell's total is Poisson (mean = variance = Lambda)."""
    wl, pl = small_plasma(T=3.0, ncell=4, ppc=64, channels=6, g_ae=1e-13, w_a=2e-37,
                          wa_mul=(1.0, 1.0, 0.08), lambda_cap=0.25, boost=1.0, dtype="f64")
    el = pl["species"]["electrons"]
    rng = np.random.default_rng(3)
    el["w"] = el["w"] * rng.lognormal(0.0, 0.5, el["w"].size)     # unequal weights
    sim = O.OracleSim(pl, wl.params)
    cells = sim.cells()
    off = el["off"]
    n = sim.el.n
    steps = 400
    counts = np.zeros((2, n))
    wsum = np.zeros((2, n))
    Ncell = []
    lam_ref = None
    for s in range(steps):
        prod, Lam, N = O.emit_thermal_cells(sim.grid, sim.params, cells, sim.el, off, s, 10 ** 9)
        for ch in (1, 2):
            m = prod["chan"] == ch
            np.add.at(counts[ch - 1], prod["parent"][m], 1)
            np.add.at(wsum[ch - 1], prod["parent"][m], prod["w"][m])
        Ncell.append(N)
        if lam_ref is None:
            lam_ref = Lam
    # per-electron means from the per-electron operator's own rates
    _, lam_e, _ = O.emit_thermal(sim.grid, sim.params, cells, sim.el, 0, 10 ** 9)
    cap = 0.25
    wprod = np.array([wl.params.w_a * wl.params.wa_mul[1], wl.params.w_a * wl.params.wa_mul[2]])
    for ch in (0, 1):
        le = np.minimum(lam_e[ch], cap)
        assert (lam_e[ch] > cap).sum() > 5                       # some electrons capped
        exp_n = steps * le
        chi2 = float(((counts[ch] - exp_n) ** 2 / exp_n).sum())
        dof = n
        assert abs(chi2 - dof) < 5 * math.sqrt(2 * dof), (ch, chi2, dof)
        # physical yield per electron: lambda_e w_prod per step, capped ones included
        yld = wsum[ch] / steps
        tot_exp = (lam_e[ch] * wprod[ch]).sum()
        assert yld.sum() == pytest.approx(tot_exp, rel=5 / math.sqrt(counts[ch].sum()))
    # the cell totals are Poisson with the cell mean
    Ncell = np.array(Ncell)                     # [steps, 2, ncell]
    for ch in (0, 1):
        L = lam_ref[ch]
        mean = Ncell[:, ch, :].mean(axis=0)
        var = Ncell[:, ch, :].var(axis=0, ddof=1)
        assert np.all(np.abs(mean - L) <= 6 * np.sqrt(L / steps)), (mean, L)
        assert np.all(np.abs(var - L) <= 6 * np.sqrt((L + 2 * L * L) / steps)), (var, L)


def test_superposed_thermal_yield_is_unbiased():
    """The superposed operator emits Q V dt per step and channel, as the per-electron one."""
    wl, pl = small_plasma(channels=6, g_ae=1e-13, w_a=4e-38, lambda_cap=math.inf, boost=1.0)
    sim = O.OracleSim(pl, wl.params)
    cells = sim.cells()
    off = pl["species"]["electrons"]["off"]
    tot = {1: [], 2: []}
    for s in range(10):
        prod, _, _ = O.emit_thermal_cells(sim.grid, sim.params, cells, sim.el, off, s, 10 ** 9)
        E = ME * np.sqrt((prod["p"] ** 2).sum(axis=0))
        for ch in (1, 2):
            m = prod["chan"] == ch
            tot[ch].append(prod["w"][m] * E[m])
    V = O.V_cell(sim.grid) * wl.ncell
    dt = O.dt_phys(sim.grid)
    c = cells[0]
    for ch, Q in ((1, c["Q_C"]), (2, c["Q_B"])):
        est = np.mean([t.sum() for t in tot[ch]]) * 1.602176634e-9 / (V * dt)
        nev = sum(t.size for t in tot[ch])
        assert nev > 2000
        assert est == pytest.approx(Q, rel=5 * 1.3 / math.sqrt(nev)), (ch, est / Q)


def test_superposed_cell_count_for_means_above_the_inversion_range():
    """A cell mean above 500 is drawn as a sum of equal Poisson parts: still Poisson."""
    wl, pl = small_plasma(T=3.0, ncell=2, ppc=64, channels=2, g_ae=1e-13, w_a=3e-39,
                          lambda_cap=math.inf, boost=1.0, dtype="f64")
    sim = O.OracleSim(pl, wl.params)
    cells = sim.cells()
    off = pl["species"]["electrons"]["off"]
    Ns, L = [], None
    for s in range(300):
        _, Lam, N = O.emit_thermal_cells(sim.grid, sim.params, cells, sim.el, off, s, 10 ** 9,
                                         counts_only=True)
        Ns.append(N[0])
        L = Lam[0]
    assert np.all(L > 1000) and np.all(L < 4000)
    Ns = np.array(Ns, dtype=np.float64)
    mean, var = Ns.mean(axis=0), Ns.var(axis=0, ddof=1)
    assert np.all(np.abs(mean - L) <= 6 * np.sqrt(L / 300)), (mean, L)
    assert np.all(np.abs(var - L) <= 6 * np.sqrt((L + 2 * L * L) / 300)), (var, L)


def _directions(prod):
    p = prod["p"]
    pm = np.sqrt((p ** 2).sum(axis=0))
    return p / pm, pm


@pytest.mark.parametrize("operator", ["particle", "cells"])
def test_thermal_emission_directions_are_isotropic(operator):
    """Secs. II.G and II.H draw emission directions isotropically.  Over more than 1e5
    products of the per-electron operator and of the per-cell superposition: unit
    directions with |p| = E / m_e c^2; <n_i> = 0 and <n_i n_j> = delta_ij / 3 within
    five standard errors (Var n_i = 1/3, Var n_i^2 = 4/45, Var n_i n_j = 1/15 for the
    uniform law on the sphere); cos(theta) uniform on [-1, 1] and phi uniform on
    [0, 2 pi) by Kolmogorov-Smirnov; cos(theta) uncorrelated with the energy.  A
    mapping such as cos(theta) = u, or phi over half the circle, fails several of these."""
    from scipy import stats as S
    wl, pl = small_plasma(T=3.0, ncell=4, ppc=2048, channels=6, g_ae=1e-13, w_a=1.5e-38,
                          lambda_cap=math.inf, boost=1.0)
    sim = O.OracleSim(pl, wl.params)
    cells = sim.cells()
    off = pl["species"]["electrons"]["off"]
    ns, es = [], []
    s = 0
    while sum(a.shape[1] for a in ns) < 120_000:
        if operator == "particle":
            prod, _, _ = O.emit_thermal(sim.grid, sim.params, cells, sim.el, s, 10 ** 9)
        else:
            prod, _, _ = O.emit_thermal_cells(sim.grid, sim.params, cells, sim.el, off, s, 10 ** 9)
        n, pm = _directions(prod)
        # the product's momentum magnitude is its sampled energy (massless, Sec. II.B)
        np.testing.assert_allclose(np.sqrt((n ** 2).sum(axis=0)), 1.0, atol=1e-14)
        ns.append(n)
        es.append(pm)
        s += 1
        assert s < 40
    n = np.concatenate(ns, axis=1)
    E = np.concatenate(es)
    N = n.shape[1]
    mean = n.mean(axis=1)
    assert np.all(np.abs(mean) < 5 * math.sqrt(1.0 / (3 * N))), mean
    M2 = (n[:, None, :] * n[None, :, :]).mean(axis=2)
    for i in range(3):
        assert abs(M2[i, i] - 1.0 / 3.0) < 5 * math.sqrt(4.0 / 45.0 / N), M2
        for j in range(i + 1, 3):
            assert abs(M2[i, j]) < 5 * math.sqrt(1.0 / 15.0 / N), M2
    mu = n[2]
    phi = np.mod(np.arctan2(n[1], n[0]), 2 * math.pi)
    assert S.kstest(mu, S.uniform(loc=-1.0, scale=2.0).cdf).pvalue > 1e-4
    assert S.kstest(phi, S.uniform(loc=0.0, scale=2 * math.pi).cdf).pvalue > 1e-4
    r = np.corrcoef(mu, E)[0, 1]
    assert abs(r) < 5 / math.sqrt(N), r
