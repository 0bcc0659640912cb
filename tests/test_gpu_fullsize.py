"""The workloads at their full sizes (needs an MI355X).

* The uniform all-channel forward plasmas, 512x512 cells with 64 particles per
  cell and species (fp32), over the grid T in {1.3, 3, 5} keV x n_e in
  {1e25, 6e25} cm^-3 x Z in {1, 2}, 500 steps each: the integrated power of
  each channel against the closed-form emissivity over the histogram range,
  and the binned spectra (App. B) bin by bin against the closed-form spectra,
  to statistical bars.
* The forward + inverse relaxation at 1024x1024 cells, 32 per cell and
  species, lognormal weights, electron-to-axion macro-weight ratio 100, FP64
  feedback with the temperature evolved: the axion number and energy reach
  the one-polarisation blackbody of the evolved temperature field and stay
  there, and the energy of electrons + photons + axions is conserved.
* The graded 3D plasma at 256^3 cells with Poisson(32) particles per cell and
  species (1.6e9 particles).

The oracle cannot run these plasmas whole, so it runs the particles of a
seeded sample of cells, taken from the input arrays with the cells
renumbered.  Every operator is cell-local: the sample's cell states (from its
own deposits), its particles' means, decisions and products and its feedback
are those of the full problem.  For each workload three links are checked:
the means the GPU materialises for the sampled parents against the oracle's
own (1e-5, FP32); the fused kernels of the step against the rate-fed path fed
those materialised means, over the whole plasma (GPU alone, bit for bit); and
seeded means handed to both sides, zero outside the sample on the GPU, so the
GPU's products are exactly those of the sampled parents, issued in the same
order with the same ids as the oracle's: counts, ids, cells and positions
bit-exact, momenta and weights to 1e-6, exchange buffers to 1e-6, then the
feedback and temperature update of the sampled cells.
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
ZETA3 = 1.2020569031595942
STATE_FIELDS = ["T", "n_e", "n_e_dep", "nZ", "nZ2", "rho", "XH", "kappa2", "G_P0", "G_C", "G_B"]


def log(msg):
    print(f"[fullsize] {msg}", flush=True)


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def host(a):
    return a.cpu().numpy() if torch.is_tensor(a) else np.asarray(a)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pick_cells(ncell, k, seed, must=()):
    rng = np.random.default_rng([seed, 0x5E1])
    sel = np.concatenate([rng.choice(ncell, k, replace=False), np.asarray(must, np.int64)])
    return np.unique(sel).astype(np.int64)


def gather(off, sel):
    """Particle indices of the cells `sel` of a cell-sorted species with offsets `off`,
    and the particles' renumbered cells 0..len(sel)-1."""
    off = host(off).astype(np.int64)
    lo = off[sel]
    cnt = off[sel + 1] - lo
    rep = np.repeat(np.arange(sel.size), cnt)
    start = np.cumsum(cnt) - cnt
    idx = lo[rep] + np.arange(int(cnt.sum())) - start[rep]
    return idx, rep.astype(np.int32), cnt


def sub_species(sp, idx, rep):
    """FP64 oracle species (physical weights) of the particles `idx` of an input species."""
    ti = torch.from_numpy(idx)

    def take(a, rows=False):
        if torch.is_tensor(a):
            t = ti.to(a.device)
            return (a[:, t] if rows else a[t]).double().cpu().numpy()
        return (a[:, idx] if rows else a[idx]).astype(np.float64)
    x = take(sp["x"], rows=True)
    p = None if sp["p"] is None else take(sp["p"], rows=True)
    w = take(sp["w"]) * sp["w_ref"]
    if sp.get("id") is not None:
        pid = host(sp["id"])[idx].astype(np.uint64)
    else:
        pid = (idx + int(sp["id0"])).astype(np.uint64)
    return O.OSpecies(x, p, w, pid, rep)


class Sample:
    """The particles of the cells `sel`, from the input arrays, as an oracle problem with
    the cells renumbered; the cell states come from the sample's own deposits."""

    def __init__(self, pl, params, sel):
        sp = pl["species"]
        self.sel, self.K, self.grid = sel, sel.size, pl["grid"]
        self.idx = {}
        sub = {}
        for name in ("electrons", "ions", "photons"):
            idx, rep, cnt = gather(sp[name]["off"], sel)
            self.idx[name] = idx
            sub[name] = sub_species(sp[name], idx, rep)
            if name == "electrons":
                self.el_off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
        self.el, self.ion, self.ph = sub["electrons"], sub["ions"], sub["photons"]
        self.params = dict(params.as_dict())
        if not self.params["w_gamma_prod"] > 0.0:
            self.params["w_gamma_prod"] = sp["photons"]["w_ref"]
        self.T = np.asarray(pl["T_cell"], dtype=np.float64)[sel].copy()
        V = O.V_cell(self.grid)
        self.cells = O.cell_state(self.grid, self.params, self.T,
                                  O.deposit(self.el, self.K, V), [O.deposit(self.ion, self.K, V)],
                                  [sp["ions"]["Z"]], [sp["ions"]["A"]])
        self.next_id = int(pl["next_id"])


def check_state(g, S):
    st = g.state.view(-1, B.STATE_N)[torch.from_numpy(S.sel).cuda()].cpu().numpy()
    for k, f in enumerate(STATE_FIELDS):
        np.testing.assert_allclose(st[:, k], S.cells[f], rtol=1e-12, atol=0, err_msg=f)


def check_means(g, S):
    """The materialised means of the sampled parents against the oracle's own."""
    ip = torch.from_numpy(S.idx["photons"]).cuda()
    ie = torch.from_numpy(S.idx["electrons"]).cuda()
    lamP = np64(g.rates(g.ph, B.PRIMAKOFF)[ip])
    _, olamP, _ = O.emit_primakoff(S.grid, S.params, S.cells, S.ph.copy(), 0, 1 << 40)
    np.testing.assert_allclose(lamP, olamP, rtol=1e-5)
    lamC = np64(g.rates(g.el, B.COMPTON)[ie])
    lamB = np64(g.rates(g.el, B.BREMS)[ie])
    _, olamT, _ = O.emit_thermal(S.grid, S.params, S.cells, S.el.copy(), 0, 1 << 40)
    np.testing.assert_allclose(lamC, olamT[0], rtol=1e-5)
    np.testing.assert_allclose(lamB, olamT[1], rtol=1e-5)
    assert olamP.max() > 0 and olamT[0].max() > 0
    log(f"means of {ip.numel()} photons and {ie.numel()} electrons in {S.K} cells match")


def check_fused(pl, params, **kw):
    """The step's fused kernels against the rate-fed path fed their materialised means,
    over the whole plasma, on the GPU alone."""
    g = AxpicSim(pl, params, **kw)
    g2 = AxpicSim(pl, params, **kw)
    lamP = g.rates(g.ph, B.PRIMAKOFF).clone()
    lamT = torch.stack([g.rates(g.el, B.COMPTON), g.rates(g.el, B.BREMS)]).contiguous()
    g.fb.zero_()
    g2.fb.zero_()
    kP, kP2 = g.emit_primakoff(), g2.emit_primakoff(lam_in=lamP)
    del lamP
    kT, kT2 = g.emit_thermal(), g2.emit_thermal(lam_in=lamT.reshape(-1))
    del lamT
    log(f"fused vs rate-fed: Primakoff {kP}/{kP2}, thermal {kT}/{kT2}")
    assert kP == kP2 and kT == kT2 and kP > 1000 and kT > 1000
    n = g.ax.n
    assert g2.ax.n == n
    for a, b in [(g.ax.w, g2.ax.w), (g.ax.id, g2.ax.id), (g.ax.cell, g2.ax.cell)] + \
            [(g.ax.x[d], g2.ax.x[d]) for d in range(g.ndim)] + \
            [(g.ax.p[d], g2.ax.p[d]) for d in range(3)]:
        assert torch.equal(a[:n], b[:n])
    assert torch.equal(g.ph.w[: g.ph.n], g2.ph.w[: g2.ph.n])
    # FP64 atomics: the summation order differs
    assert bool(((g.fb - g2.fb).abs() <= 1e-12 * g2.fb.abs()).all())


def compare_products(gsp, n0, prod, sel, exact_p, rtol=1e-6):
    n = prod["w"].size
    assert gsp.n - n0 == n
    sl = slice(n0, n0 + n)
    np.testing.assert_array_equal(gsp.id[sl].cpu().numpy().view(np.uint64), prod["id"])
    np.testing.assert_array_equal(gsp.cell[sl].cpu().numpy(), sel[prod["cell"]])
    for d in range(gsp.ndim):
        np.testing.assert_array_equal(np64(gsp.x[d][sl]), prod["x"][d])
    gp = np.stack([np64(gsp.p[d][sl]) for d in range(3)])
    if exact_p:
        np.testing.assert_array_equal(gp, prod["p"])
    else:
        np.testing.assert_allclose(gp, prod["p"], rtol=rtol, atol=rtol * np.abs(prod["p"]).max())
    np.testing.assert_allclose(np64(gsp.w[sl]) * gsp.w_ref, prod["w"], rtol=rtol)


def scatter(n, idx, vals, rows=1):
    """A device array of n means (per row) that holds `vals` at `idx` and zero elsewhere."""
    dt = torch.float32 if vals.dtype == np.float32 else torch.float64
    out = torch.zeros((rows, n), dtype=dt, device="cuda")
    out[:, torch.from_numpy(idx).cuda()] = dev(vals.reshape(rows, -1))
    return out.reshape(-1) if rows == 1 else out


def seeded_chain(g, S, seed, axd=None, feedback=False):
    """Rate-fed Primakoff, thermal emission and (given a seeded axion population)
    absorption + a->gamma on the sampled parents, against the oracle's run of the
    sample; then the feedback and temperature update of the sampled cells."""
    sel = S.sel
    sdev = torch.from_numpy(sel).cuda()
    g.fb.zero_()
    fb = np.zeros(S.K * 4)
    oid = g.next_id
    if axd is not None:
        ia, rep, _ = gather(axd["off"], sel)
        oax = sub_species(axd, ia, rep)
        n_old = g.ax.n
        assert n_old == axd["n"] and oid == axd["next_id"]
    # Primakoff
    ip = S.idx["photons"]
    lamP = I.means(ip.size, seed=seed, lo=1e-5, hi=2.0)
    n0 = g.ax.n
    kP = g.emit_primakoff(lam_in=scatter(g.ph.n, ip, lamP))
    prod, _, _ = O.emit_primakoff(S.grid, S.params, S.cells, S.ph, 0, oid,
                                  lam_in=lamP.astype(np.float64))
    log(f"seeded Primakoff: {kP} events from {ip.size} sampled photons")
    assert kP == prod["w"].size and kP > 100
    compare_products(g.ax, n0, prod, sel, exact_p=True)
    np.testing.assert_allclose(np64(g.ph.w[torch.from_numpy(ip).cuda()]) * g.ph.w_ref, S.ph.w,
                               rtol=1e-6)
    oid += prod["w"].size
    # thermal emission
    ie = S.idx["electrons"]
    lamT = I.means(ie.size, seed=seed + 1, rows=2, lo=1e-5, hi=0.5)
    n0 = g.ax.n
    kT = g.emit_thermal(lam_in=scatter(g.el.n, ie, lamT, rows=2).reshape(-1))
    prod, _, _ = O.emit_thermal(S.grid, S.params, S.cells, S.el, 0, oid, fb,
                                lam_in=lamT.astype(np.float64))
    log(f"seeded thermal emission: {kT} events from {ie.size} sampled electrons")
    assert kT == prod["w"].size and kT > 100
    compare_products(g.ax, n0, prod, sel, exact_p=False)
    oid += prod["w"].size
    # absorption and a->gamma of the seeded axions of the sampled cells
    if axd is not None:
        pab = I.means(ia.size, seed=seed + 2, lo=1e-5, hi=0.6)
        lag = I.means(ia.size, seed=seed + 3, lo=1e-4, hi=2.0)
        ph0 = g.ph.n
        k = g.absorb(n_old, pabs_in=scatter(n_old, ia, pab), lam_in=scatter(n_old, ia, lag))
        prod, _, _, _, dead = O.absorb(S.grid, S.params, S.cells, oax, 0, oid, fb,
                                       pabs_in=pab.astype(np.float64),
                                       lam_in=lag.astype(np.float64))
        log(f"seeded absorption: {int(dead.sum())} absorbed, {k} a->gamma photons from "
            f"{ia.size} sampled axions")
        assert k == prod["w"].size and k > 20 and dead.sum() > 10
        compare_products(g.ph, ph0, prod, sel, exact_p=False)
        gw = np64(g.ax.w[torch.from_numpy(ia).cuda()]) * g.ax.w_ref
        np.testing.assert_array_equal(gw == 0.0, oax.w == 0.0)
        np.testing.assert_allclose(gw, oax.w, rtol=2e-6, atol=0)
    torch.cuda.synchronize()
    gfb = g.fb.view(-1, 4)[sdev].cpu().numpy().reshape(-1)
    np.testing.assert_allclose(gfb, fb, rtol=1e-6, atol=1e-9 * np.abs(fb).max())
    if feedback:
        g.feedback()
        O.feedback(S.grid, S.params, S.el_off, S.el, fb, S.T)
        torch.cuda.synchronize()
        ie_d = torch.from_numpy(ie).cuda()
        gp = np.stack([np64(g.el.p[d][ie_d]) for d in range(3)])
        np.testing.assert_allclose(gp, S.el.p, rtol=2e-6, atol=2e-6 * np.abs(S.el.p).max())
        np.testing.assert_allclose(g.T[sdev].cpu().numpy(), S.T, rtol=1e-7)
        log(f"feedback and temperature of {S.K} sampled cells match")


# ---------------------------------------------------------------------------
# uniform all-channel forward plasmas, 512x512 x 64 per cell and species
# ---------------------------------------------------------------------------
GRID = [(T, ne, Z) for T in (1.3, 3.0, 5.0) for ne in (1e25, 6e25) for Z in (1, 2)]


def _closed_forms(wl):
    c0 = O.cell_state(wl.grid(), wl.params, np.array([wl.T_keV]), np.array([wl.n_e]),
                      [np.array([wl.n_e / wl.Z])], [float(wl.Z)], [wl.A])[0]
    return c0, [A.dQdE_primakoff, A.dQdE_compton, A.dQdE_brems]


def _photon_fractions(edges, T):
    """Fraction of blackbody photons in each histogram bin (closed-form total density
    2 zeta(3) T^3 / (pi^2 (hbar c)^3))."""
    from scipy import integrate
    tot = 2.0 * ZETA3 * T ** 3 / (math.pi ** 2 * HBARC ** 3)
    f = lambda x: float(A.dn_blackbody(np.array([x]), T)[0])
    return np.array([integrate.quad(f, edges[k], edges[k + 1], epsrel=1e-10)[0]
                     for k in range(edges.size - 1)]) / tot


@pytest.mark.parametrize("T,ne,Z", GRID, ids=[f"T{t}-ne{n:.0e}-Z{z}" for t, n, z in GRID])
def test_forward_plasma_grid_power_and_spectra(T, ne, Z):
    """Each plasma is run for its full 500 steps (seeds 0..11 over the grid).  The bars
    are statistical: the compound-Poisson variance of the macro-events of each bin
    (every event adds w E with E below the bin's upper edge, so sigma^2 <= w E_hi X), plus,
    for Primakoff, the sampling variance of the frozen photon population in the bin
    (multinomial, relative variance 1 / N_photons in the bin)."""
    seed = GRID.index((T, ne, Z))
    wl = I.config2(T_keV=T, n_e=ne, Z=Z, seed=seed)
    log(f"forward plasma T={T} n_e={ne:.0e} Z={Z} n={wl.n} ppc={wl.ppc} seed={seed}")
    c0, fns = _closed_forms(wl)
    lo, hi = wl.params.hist_lo_keV, wl.params.hist_hi_keV
    V = wl.ncell * wl.V_cell_cm3
    dtp = wl.dt / wl.omega0
    # closed-form powers over the histogram range; product weights sized for about 5e4
    # macro-events per channel and step
    Q = [A.integrate_Q(fn, lo, hi, c0, wl.params) for fn in fns]
    meanE = [3.0 * T, c0["meanE_C"], c0["meanE_B"]]
    rate = [q / (e * KEV_ERG) * V * dtp for q, e in zip(Q, meanE)]
    assert min(Q) > 0.0
    wl.params.wa_mul = tuple(r / (wl.params.w_a * 5e4) for r in rate)
    pl = I.make_plasma_device(wl, seed)
    sel = pick_cells(wl.ncell, 64, seed=seed, must=(0, wl.ncell - 1))
    S = Sample(pl, wl.params, sel)
    g = AxpicSim(pl, wl.params)
    check_state(g, S)
    check_means(g, S)
    del g
    check_fused(pl, wl.params)
    g = AxpicSim(pl, wl.params)
    seeded_chain(g, S, seed=70 + seed)
    del g
    g = AxpicSim(pl, wl.params, axion_capacity=int(1.6e8))
    n_ph = pl["species"]["photons"]["n"]
    del pl
    steps = wl.steps
    for s in range(steps):
        g.step()
        if s % 100 == 99:
            log(f"step {s + 1}: {g.ax.n} axions")
    h = g.hist_np()
    nb = wl.params.hist_nbins
    e = A.hist_edges(wl.params)
    t_tot = steps * dtp
    Nph = n_ph * _photon_fractions(e, T)
    for i, fn in enumerate(fns):
        Qmc = h[i][:nb].sum() * KEV_ERG / (V * t_tot)
        wprod = wl.params.w_a * wl.params.wa_mul[i]
        X = A.binned_expectation(fn, wl.params, c0, wl.params) * V * t_tot / KEV_ERG
        var = wprod * e[1:] * X
        if i == 0:
            var = var + X * X / np.maximum(Nph, 1.0)
        sQ = math.sqrt(var.sum()) / X.sum()
        ev = X / (wprod * np.sqrt(e[:-1] * e[1:]))
        use = ev > 30.0
        z = (h[i][:nb] - X)[use] / np.sqrt(var[use])
        chi2 = float((z * z).mean())
        log(f"channel {i}: power MC / closed form {Qmc / Q[i]:.6f} (sigma {sQ:.1e}), "
            f"{int(use.sum())} bins, max |z| {np.abs(z).max():.2f}, chi2/bin {chi2:.3f}")
        assert abs(Qmc / Q[i] - 1.0) < 5.0 * sQ + 1e-4, i
        assert use.sum() >= 40
        assert np.abs(z).max() < 5.5, i
        assert chi2 < 1.6, i


# ---------------------------------------------------------------------------
# forward + inverse relaxation, 1024x1024 x 32 per cell and species
# ---------------------------------------------------------------------------
def _energy(g):
    """FP64 energies [keV x physical count] of electrons (kinetic, non-relativistic),
    photons and axions."""
    def kin(sp):
        return sum(sp.p[d][: sp.n].double() ** 2 for d in range(3))
    Ee = 0.5 * ME * float((g.el.w[: g.el.n].double() * kin(g.el)).sum()) * g.el.w_ref
    Eg = ME * float((g.ph.w[: g.ph.n].double() * kin(g.ph).sqrt()).sum()) * g.ph.w_ref
    Ea = ME * float((g.ax.w[: g.ax.n].double() * kin(g.ax).sqrt()).sum()) * g.ax.w_ref
    Na = float(g.ax.w[: g.ax.n].double().sum()) * g.ax.w_ref
    return Ee, Eg, Ea, Na


@pytest.mark.parametrize("ratio", [1.0, 10.0, 100.0])
def test_relaxation_full_size_reaches_blackbody_and_conserves_energy(ratio):
    """Electron-to-axion macro-weight ratios 1, 10 and 100; the oracle chain on sampled
    cells runs at ratio 100, where the axions are lightest and most numerous."""
    wl = I.config3(ratio=ratio)
    log(f"relaxation n={wl.n} ppc={wl.ppc} ratio {ratio:g} lognormal sigma "
        f"{wl.lognormal_sigma}")
    pl = I.make_plasma_device(wl, 0)
    if ratio == 100.0:
        sel = pick_cells(wl.ncell, 256, seed=3, must=(0, wl.ncell - 1))
        S = Sample(pl, wl.params, sel)
        g = AxpicSim(pl, wl.params)
        check_state(g, S)
        check_means(g, S)
        del g
        check_fused(pl, wl.params)
        g = AxpicSim(pl, wl.params)
        axd = I.make_axions(wl, pl, 8.0, seed=5)
        g.load_axions(axd, extra=1 << 20)
        seeded_chain(g, S, seed=80, axd=axd, feedback=True)
        del g, axd
    g = AxpicSim(pl, wl.params, axion_capacity=int(4e5 * ratio) + (1 << 20), compact_every=16)
    del pl
    V_cell = wl.V_cell_cm3
    Ee0, Eg0, _, _ = _energy(g)
    E0 = Ee0 + Eg0
    steps = wl.steps
    rec = []
    for s in range(1, steps + 1):
        g.step()
        if s % 100 == 0:
            Ee, Eg, Ea, Na = _energy(g)
            T = g.T.double()
            # the library's FP64 equilibrium check at the evolved temperature field; its
            # totals are the one-state blackbody zeta(3) T^3/pi^2, pi^2 T^4/30 per cell
            eq = g.equilibrium(t_steps=s)
            Neq, Ueq = float(eq["neq"].sum()), float(eq["ueq"].sum())
            assert Neq == pytest.approx(float((T ** 3).sum()) * ZETA3 /
                                        (math.pi ** 2 * HBARC ** 3) * V_cell, rel=1e-7)
            assert Ueq == pytest.approx(float((T ** 4).sum()) * math.pi ** 2 /
                                        (30.0 * HBARC ** 3) * V_cell, rel=1e-7)
            assert float(eq["num"].sum()) == pytest.approx(Na, rel=1e-9)
            if s == steps:
                band = (eq["nfix"] > 1e-3 * eq["nfix"].max())
                band[-2:] = False
                log(f"step {s}: per-bin axion number / recursion content "
                    f"{np.round(eq['num'][band] / eq['nfix'][band], 3)}")
            d = g.diag()
            rec.append((s, Na / Neq, Ea / Ueq, (Ee + Eg + Ea) / E0 - 1.0, Na))
            log(f"step {s}: N_a/N_eq {Na / Neq:.4f}, U_a/U_eq {Ea / Ueq:.4f}, "
                f"energy drift {rec[-1][3]:+.2e}, mean T {float(T.mean()):.4f} keV, "
                f"axions {g.ax.n}, photon energy {Eg / Eg0 - 1.0:+.4f}")
            assert d["N_a"] == pytest.approx(Na, rel=1e-9)
            assert d["U_a"] == pytest.approx(Ea, rel=1e-9)
            assert abs(rec[-1][3]) < 1e-6
    st = g.stats_dict()
    assert st["clamped_cells"] == 0 and st["cold_cells"] == 0
    last = [r for r in rec if r[0] > 0.75 * steps]
    prev = [r for r in rec if 0.5 * steps < r[0] <= 0.75 * steps]
    for r in last:
        assert r[1] == pytest.approx(1.0, abs=0.02)
        assert r[2] == pytest.approx(1.0, abs=0.025)
    drift = np.mean([r[4] for r in last]) / np.mean([r[4] for r in prev]) - 1.0
    log(f"axion number, last quarter over the quarter before: {drift:+.4f}")
    assert abs(drift) < 0.01


# ---------------------------------------------------------------------------
# graded 3D plasma, 256^3 x Poisson(32) per cell and species
# ---------------------------------------------------------------------------
def test_graded_plasma_full_size_sampled_cells():
    wl = I.config5()
    log(f"graded plasma n={wl.n} Poisson ppc={wl.ppc}")
    pl = I.make_plasma_device(wl, 0)
    nx = wl.n[0]
    # cells at both ends of the gradient and a seeded spread in between
    sel = pick_cells(wl.ncell, 256, seed=5, must=(0, nx - 1, wl.ncell - nx, wl.ncell - 1))
    S = Sample(pl, wl.params, sel)
    assert S.T.min() < 1.1 and S.T.max() > 4.9
    log(f"sample: {S.K} cells, {S.el.n} electrons, {S.ph.n} photons")
    g = AxpicSim(pl, wl.params)
    check_state(g, S)
    check_means(g, S)
    del g
    torch.cuda.empty_cache()
    check_fused(pl, wl.params)
    torch.cuda.empty_cache()
    g = AxpicSim(pl, wl.params)
    axd = I.make_axions(wl, pl, 2.0, seed=6)
    g.load_axions(axd, extra=1 << 24)
    del pl
    seeded_chain(g, S, seed=90, axd=axd, feedback=True)
