"""Seeded synthetic workloads for the axion Monte-Carlo operators.

This module builds the *inputs* of a run: the grid scale, the static plasma
macroparticles (electrons, ions, blackbody photons) and the method's
user parameters.  It contains none of the method's arithmetic (no rates, no
sampling of emission events, no feedback); both the HIP path and the FP64
oracle consume what it returns.

Workload recipe (uniform static thermal plasma, the benchmark setting of
Sec. III.A of the paper, extended to the five workloads the hot path is
measured on):

* grid: ``ndim`` periodic dimensions of ``n`` cells; cell size ``dx = 0.2``
  and step ``dt = 0.1`` in the PIC normalisation (length c/omega0, time
  1/omega0), ``omega0`` = electron plasma frequency at the reference density.
  Transverse extents of 1D/2D grids are one cell size, so every cell has the
  volume ``(dx c/omega0)^3``.
* electrons: non-relativistic Maxwellian momenta, every component normal with
  variance ``T/(m_e c^2)`` (momentum in units of m_e c).
* ions: static, one species (Z, A); momenta are not stored (deposit-only).
* photons: blackbody energies ``x = omega/T`` drawn from ``x^2/(e^x-1)`` by its
  exact mixture representation (``x = Gamma(3)/j`` with ``j`` distributed as
  ``j^-3/zeta(3)``), isotropic directions.  Their physical density is the
  blackbody number density ``2 zeta(3) T^3 / (pi^2 (hbar c)^3)``.
* positions: uniform inside the cell, stored in cell units; particles are
  grouped by cell in cell order (so every species starts cell-sorted).
* weights: relative weights ``w~`` (physical weight = ``w_ref * w~``), either
  all one or lognormal with sigma 0.5 normalised to unit mean.
* per-cell counts: fixed ``ppc`` or Poisson with mean ``ppc``.
* graded plasmas: temperature and density linear in x; the density grading
  is carried by the relative weights of the cell's particles.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import Dict, Optional

import numpy as np

# Physical constants used only to set up the workload (CODATA 2018, cgs / keV).
_ME_KEV = 510.99895000
_HBARC_KEVCM = 1.973269804e-8
_ZETA3 = 1.2020569031595942854
_C_CMS = 2.99792458e10
_WPE_COEF = 5.64146e4  # sqrt(4 pi e^2 / m_e) in cgs: omega_pe = _WPE_COEF * sqrt(n_e)

KIND_ELECTRON, KIND_ION, KIND_PHOTON, KIND_AXION = 0, 1, 2, 3

CH_PRIMAKOFF, CH_COMPTON, CH_BREMS = 1, 2, 4


@dataclass
class Params:
    """User parameters of the method (plain data, shared by both sides)."""
    g_agg_GeV: float = 1e-10          # axion-photon coupling [GeV^-1]
    g_ae: float = 1e-13               # axion-electron coupling
    channels: int = CH_PRIMAKOFF      # bitmask of active forward channels
    inverse: int = 0                  # 1: inverse operators (absorption, a->gamma) on
    w_a: float = 1e-36                # axion macro-weight (physical axions per macroparticle)
    wa_mul: tuple = (1.0, 1.0, 1.0)   # product base weight multipliers (Primakoff, Compton, brems)
    w_gamma_prod: float = 0.0         # photon product weight for a->gamma (0: photon w_ref)
    lambda_cap: float = math.inf      # Poisson-mean cap
    boost: float = 1.0                # common multiplier of every rate (relaxation studies)
    eq_stats: int = 0                 # 0 Bose-Einstein, 1 Maxwell-Boltzmann
    kappa_mode: int = 0               # 0 Debye from deposits, 1 fixed
    kappa_fixed_keV: float = 0.0
    prim_targets: int = 0             # 0 sum Z_i^2 n_i over ions, 1 include electrons (n_eff)
    prim_inv_ratio: float = 1.0       # Gamma(a->gamma) / Gamma(gamma->a)
    brems_ee: int = 1                 # include the electron-electron term
    brems_k: float = 1.70             # Gamma-sampler shape
    brems_theta: float = 1.0          # Gamma-sampler scale (in units of T)
    absorb_mode: int = 0              # 0 Bernoulli deletion, 1 weight reduction
    quasi_neutral: int = 0            # n_e from sum Z_i n_i instead of deposited electrons
    T_mode: int = 0                   # 0 fixed, 1 prescribed field, 2 evolved by feedback
    feedback: int = 0                 # apply the affine remap from the exchange buffers
    r_relax: float = 0.1
    T_floor_keV: float = 0.05
    T_ceil_keV: float = 100.0
    seed: int = 0
    hist_lo_keV: float = 0.1
    hist_hi_keV: float = 20.0
    hist_nbins: int = 128
    hist_log: int = 1
    m_a_keV: float = 0.0              # axion mass (0: massless, the paper's validated case)
    light_mode: int = 0               # parents lighter than the product weight: 0 convert whole
                                      # with probability P, 1 literal Poisson count

    def as_dict(self) -> Dict:
        return asdict(self)


@dataclass
class Workload:
    name: str
    ndim: int
    n: tuple
    ppc: int
    dtype: str                      # "f32" or "f64"
    T_keV: float                    # uniform temperature (or x=0 end of a grading)
    n_e: float                      # electron density [cm^-3] (or x=0 end)
    Z: int = 1
    A: float = 1.0
    T_keV_hi: Optional[float] = None   # graded plasma: value at x = L
    n_e_hi: Optional[float] = None
    poisson_ppc: bool = False
    lognormal_sigma: float = 0.0
    dx: float = 0.2
    dt: float = 0.1
    n_ref: Optional[float] = None   # density defining omega0 (default: n_e)
    steps: int = 100
    params: Params = field(default_factory=Params)

    @property
    def ncell(self) -> int:
        return int(np.prod(self.n))

    @property
    def omega0(self) -> float:
        nref = self.n_ref if self.n_ref is not None else self.n_e
        return _WPE_COEF * math.sqrt(nref)

    @property
    def V_cell_cm3(self) -> float:
        return (self.dx * _C_CMS / self.omega0) ** 3

    def grid(self) -> Dict:
        n = tuple(self.n) + (1,) * (3 - len(self.n))
        return dict(ndim=self.ndim, n=n, dx=self.dx, dt=self.dt, omega0=self.omega0)


def blackbody_density(T_keV: float) -> float:
    """Photon number density of a blackbody at T [cm^-3]."""
    return 2.0 * _ZETA3 * T_keV ** 3 / (math.pi ** 2 * _HBARC_KEVCM ** 3)


def _cell_profile(wl: Workload):
    """Per-cell temperature [keV] and electron density [cm^-3] (graded along x)."""
    nx = wl.n[0]
    xc = (np.arange(nx) + 0.5) / nx
    T_hi = wl.T_keV if wl.T_keV_hi is None else wl.T_keV_hi
    ne_hi = wl.n_e if wl.n_e_hi is None else wl.n_e_hi
    Tx = wl.T_keV + (T_hi - wl.T_keV) * xc
    nex = wl.n_e + (ne_hi - wl.n_e) * xc
    reps = wl.ncell // nx
    # cell index = ix + nx*(iy + ny*iz): x varies fastest
    return np.tile(Tx, reps), np.tile(nex, reps)


def _counts(wl: Workload, rng: np.random.Generator) -> np.ndarray:
    if wl.poisson_ppc:
        return rng.poisson(wl.ppc, wl.ncell).astype(np.int64)
    return np.full(wl.ncell, wl.ppc, dtype=np.int64)


def _positions(wl: Workload, counts: np.ndarray, rng, dt) -> np.ndarray:
    ncell = wl.ncell
    cell = np.repeat(np.arange(ncell, dtype=np.int64), counts)
    N = cell.size
    nfull = tuple(wl.n) + (1,) * (3 - len(wl.n))
    idx = [cell % nfull[0], (cell // nfull[0]) % nfull[1], cell // (nfull[0] * nfull[1])]
    x = np.zeros((3, N), dtype=dt)
    for d in range(wl.ndim):
        u = rng.random(N)
        x[d] = (idx[d] + u).astype(dt)
        # rounding to float32 may land exactly on the upper cell face
        bad = np.floor(x[d]) != idx[d]
        if bad.any():
            x[d][bad] = np.nextafter(dt(idx[d][bad] + 1), dt(0))
    return x, cell.astype(np.int32)


def _isotropic(rng, N):
    mu = 2.0 * rng.random(N) - 1.0
    phi = 2.0 * math.pi * rng.random(N)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return np.stack([s * np.cos(phi), s * np.sin(phi), mu])


def _blackbody_x(rng, N):
    """x = omega/T with density x^2/(e^x - 1)/(2 zeta(3))."""
    J = 20000
    j = np.arange(1, J + 1, dtype=np.float64)
    pj = j ** -3
    pj /= pj.sum()
    jj = rng.choice(J, size=N, p=pj) + 1
    return rng.gamma(3.0, 1.0, N) / jj


def _weights(wl: Workload, N, rng, dt):
    if wl.lognormal_sigma > 0:
        s = wl.lognormal_sigma
        return np.exp(s * rng.standard_normal(N) - 0.5 * s * s).astype(dt)
    return np.ones(N, dtype=dt)


def make_plasma(wl: Workload, seed: Optional[int] = None) -> Dict:
    """Build the static species of a workload.

    Returns ``{"grid": ..., "species": {name: arrays}, "T_cell": [ncell]}``.
    Each species dict has ``x`` [3,N] (cell units), ``p`` [3,N] (m_e c,
    absent for ions), ``w`` [N] relative weights, ``id`` [N] uint64,
    ``cell`` [N] int32, ``off`` [ncell+1] int64 (cell offsets), and the scalars
    ``w_ref``, ``kind``, ``Z``, ``A``.
    """
    seed = wl.params.seed if seed is None else seed
    dt = np.float64 if wl.dtype == "f64" else np.float32
    ss = np.random.SeedSequence([seed, 0xA710])
    rng_e, rng_i, rng_g = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]
    T_cell, ne_cell = _cell_profile(wl)
    V = wl.V_cell_cm3
    ncell = wl.ncell
    graded = (wl.T_keV_hi is not None) or (wl.n_e_hi is not None)

    species = {}
    id_base = 0
    for name, rng in (("electrons", rng_e), ("ions", rng_i), ("photons", rng_g)):
        counts = _counts(wl, rng)
        x, cell = _positions(wl, counts, rng, dt)
        N = cell.size
        w = _weights(wl, N, rng, dt)
        c64 = cell.astype(np.int64)
        if name == "electrons":
            kind, Z, A = KIND_ELECTRON, -1.0, 0.0
            w_ref = wl.n_e * V / wl.ppc
            dens_scale = ne_cell / wl.n_e
            sig = np.sqrt(T_cell / _ME_KEV)[c64]
            p = rng.standard_normal((3, N)) * sig
        elif name == "ions":
            kind, Z, A = KIND_ION, float(wl.Z), float(wl.A)
            w_ref = wl.n_e / wl.Z * V / wl.ppc
            dens_scale = ne_cell / wl.n_e
            p = None
        else:
            kind, Z, A = KIND_PHOTON, 0.0, 0.0
            w_ref = blackbody_density(wl.T_keV) * V / wl.ppc
            dens_scale = (T_cell / wl.T_keV) ** 3
            om = _blackbody_x(rng, N) * T_cell[c64] / _ME_KEV
            p = _isotropic(rng, N) * om
        if graded:
            w = (w * dens_scale[c64]).astype(dt)
        off = np.zeros(ncell + 1, dtype=np.int64)
        np.cumsum(counts, out=off[1:])
        sp = dict(x=x, p=None if p is None else p.astype(dt), w=w,
                  id=(np.arange(N, dtype=np.uint64) + np.uint64(id_base)),
                  cell=cell, off=off, w_ref=float(w_ref), kind=kind, Z=Z, A=A, n=N)
        id_base += N
        species[name] = sp
    return dict(grid=wl.grid(), species=species, T_cell=T_cell.astype(np.float64),
                next_id=id_base)


def make_axions(wl: Workload, plasma: Dict, per_cell: float, seed: int,
                zero_frac: float = 0.02) -> Dict:
    """A seeded axion population for operator tests, built from inputs only.

    Poisson(per_cell) axions per cell, grouped by cell; positions uniform in
    the cell; energies x T_cell with x drawn from the blackbody shape
    x^2/(e^x-1) (the massless equilibrium spectrum); isotropic directions;
    lognormal relative weights (sigma 0.5, unit mean) of which a fraction
    zero_frac is exactly zero (dead axions); w_ref = the parameters' w_a; ids
    continue from plasma["next_id"].  Same keys as a make_plasma species, plus
    next_id (the first id after these)."""
    dt = np.float64 if wl.dtype == "f64" else np.float32
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0xA7A7])))
    counts = rng.poisson(per_cell, wl.ncell).astype(np.int64)
    x, cell = _positions(wl, counts, rng, dt)
    N = cell.size
    T_cell = plasma["T_cell"]
    om = _blackbody_x(rng, N) * T_cell[cell.astype(np.int64)] / _ME_KEV
    p = (_isotropic(rng, N) * om).astype(dt)
    w = np.exp(0.5 * rng.standard_normal(N) - 0.125)
    w[rng.random(N) < zero_frac] = 0.0
    off = np.zeros(wl.ncell + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    id0 = int(plasma["next_id"])
    return dict(x=x, p=p, w=w.astype(dt), id=np.arange(N, dtype=np.uint64) + np.uint64(id0),
                cell=cell, off=off, w_ref=float(wl.params.w_a), kind=KIND_AXION, Z=0.0, A=0.0,
                n=N, next_id=id0 + N)


def means(n: int, seed: int, rows: int = 1, lo: float = 1e-4, hi: float = 3.0,
          zero_frac: float = 0.02, dtype: str = "f32") -> np.ndarray:
    """Seeded Poisson means for the rate-fed sampling calls: log-uniform in
    [lo, hi], a fraction zero_frac exactly zero; shape (rows, n) (or (n,) when
    rows is 1), in the workload's storage type."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x1A3B, rows])))
    lam = np.exp(rng.uniform(math.log(lo), math.log(hi), (rows, n)))
    lam[rng.random((rows, n)) < zero_frac] = 0.0
    lam = lam.astype(np.float64 if dtype == "f64" else np.float32)
    return lam[0] if rows == 1 else lam


def make_plasma_device(wl: Workload, seed: Optional[int] = None, device="cuda") -> Dict:
    """The workload recipe of make_plasma drawn with torch's generator on the
    GPU, for plasmas too large to build on the host (the 256^3 graded plasma
    holds 1.6e9 particles).  Same layout and distributions; the random streams
    differ from make_plasma's, so it serves measurements, not oracle
    comparisons.  Arrays are device tensors; ids are implicit (``id0`` + i)."""
    import torch
    seed = wl.params.seed if seed is None else seed
    dev = torch.device(device)
    td = torch.float64 if wl.dtype == "f64" else torch.float32
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed) * 1000003 + 0xA710)
    T_np, ne_np = _cell_profile(wl)
    T_cell = torch.from_numpy(T_np).to(dev)
    ne_cell = torch.from_numpy(ne_np).to(dev)
    V = wl.V_cell_cm3
    ncell = wl.ncell
    nfull = tuple(wl.n) + (1,) * (3 - len(wl.n))
    graded = (wl.T_keV_hi is not None) or (wl.n_e_hi is not None)
    # blackbody mixture weights p_j ~ j^-3 (x = Gamma(3, 1) / j)
    J = 20000
    pj = torch.arange(1, J + 1, device=dev, dtype=torch.float64) ** -3
    cdf = torch.cumsum(pj / pj.sum(), 0)
    species = {}
    id_base = 0
    for name in ("electrons", "ions", "photons"):
        if wl.poisson_ppc:
            counts = torch.poisson(torch.full((ncell,), float(wl.ppc), device=dev,
                                              dtype=torch.float64), generator=gen).to(torch.int64)
        else:
            counts = torch.full((ncell,), wl.ppc, device=dev, dtype=torch.int64)
        cell = torch.repeat_interleave(torch.arange(ncell, device=dev, dtype=torch.int64), counts)
        N = int(cell.numel())
        x = torch.zeros((3, N), device=dev, dtype=td)
        idx = [cell % nfull[0], (cell // nfull[0]) % nfull[1], cell // (nfull[0] * nfull[1])]
        for d in range(wl.ndim):
            xd = (idx[d].to(torch.float64) + torch.rand(N, device=dev, generator=gen,
                                                        dtype=torch.float64)).to(td)
            top = torch.nextafter((idx[d] + 1).to(td), torch.zeros((), device=dev, dtype=td))
            x[d] = torch.where(torch.floor(xd) != idx[d].to(td), top, xd)
            del xd, top
        del idx
        if wl.lognormal_sigma > 0:
            sg = wl.lognormal_sigma
            w = torch.exp(sg * torch.randn(N, device=dev, generator=gen) - 0.5 * sg * sg).to(td)
        else:
            w = torch.ones(N, device=dev, dtype=td)
        p = None
        if name == "electrons":
            kind, Z, A = KIND_ELECTRON, -1.0, 0.0
            w_ref = wl.n_e * V / wl.ppc
            dens_scale = ne_cell / wl.n_e
            sig = torch.sqrt(T_cell / _ME_KEV)[cell]
            p = (torch.randn((3, N), device=dev, generator=gen, dtype=torch.float64) * sig).to(td)
            del sig
        elif name == "ions":
            kind, Z, A = KIND_ION, float(wl.Z), float(wl.A)
            w_ref = wl.n_e / wl.Z * V / wl.ppc
            dens_scale = ne_cell / wl.n_e
        else:
            kind, Z, A = KIND_PHOTON, 0.0, 0.0
            w_ref = blackbody_density(wl.T_keV) * V / wl.ppc
            dens_scale = (T_cell / wl.T_keV) ** 3
            jj = torch.searchsorted(cdf, torch.rand(N, device=dev, generator=gen,
                                                    dtype=torch.float64)).clamp_(max=J - 1) + 1
            g3 = -torch.log(torch.rand((3, N), device=dev, generator=gen,
                                       dtype=torch.float64).clamp_(min=1e-300)).sum(0)
            om = g3 / jj * T_cell[cell] / _ME_KEV
            del jj, g3
            mu = 2.0 * torch.rand(N, device=dev, generator=gen, dtype=torch.float64) - 1.0
            phi = 2.0 * math.pi * torch.rand(N, device=dev, generator=gen, dtype=torch.float64)
            sn = torch.sqrt(torch.clamp(1.0 - mu * mu, min=0.0))
            p = torch.stack([sn * torch.cos(phi) * om, sn * torch.sin(phi) * om, mu * om]).to(td)
            del mu, phi, sn, om
        if graded:
            w = (w.to(torch.float64) * dens_scale[cell]).to(td)
        off = torch.zeros(ncell + 1, device=dev, dtype=torch.int64)
        off[1:] = torch.cumsum(counts, 0)
        species[name] = dict(x=x, p=p, w=w, id=None, id0=id_base, cell=cell.to(torch.int32),
                             off=off, w_ref=float(w_ref), kind=kind, Z=Z, A=A, n=N)
        del cell, counts
        id_base += N
    return dict(grid=wl.grid(), species=species, T_cell=T_np.astype(np.float64), next_id=id_base)


# ---------------------------------------------------------------------------
# The five workloads.  Method parameters that the workload descriptions leave
# open (axion macro-weight, cap, boost) are fixed here as plain numbers.
# ---------------------------------------------------------------------------

def config1(**kw) -> Workload:
    """1D periodic, 64 cells, 64 e/ion/photon per cell, fp64, Primakoff forward,
    T = 1.3 keV, n_e = 6e25 cm^-3, g_agg = 1e-10 GeV^-1, 100 steps, seed 0,
    128 log bins over 0.1-20 keV."""
    p = Params(g_agg_GeV=1e-10, channels=CH_PRIMAKOFF, w_a=1e-36, lambda_cap=math.inf,
               seed=0, hist_lo_keV=0.1, hist_hi_keV=20.0, hist_nbins=128, hist_log=1)
    wl = Workload("cfg1", ndim=1, n=(64,), ppc=64, dtype="f64", T_keV=1.3, n_e=6e25,
                  Z=1, A=1.0, steps=100, params=p)
    for k, v in kw.items():
        setattr(wl, k, v)
    return wl


def config2(T_keV=3.0, n_e=6e25, Z=1, n=(512, 512), ppc=64, seed=0, **kw) -> Workload:
    """2D 512x512, 64 per cell per species, fp32, all three channels forward,
    g_ae = 1e-13, g_agg = 1e-10, 500 steps.  Product weights put the mean
    macro-event count near 2e-3 per particle and channel at T = 3 keV,
    n_e = 6e25 cm^-3."""
    A = 1.0 if Z == 1 else 4.0
    p = Params(g_agg_GeV=1e-10, g_ae=1e-13, channels=CH_PRIMAKOFF | CH_COMPTON | CH_BREMS,
               w_a=1e-34, wa_mul=(400.0, 1.0, 0.3), lambda_cap=16.0, seed=seed,
               hist_lo_keV=0.1, hist_hi_keV=80.0, hist_nbins=128, hist_log=1)
    wl = Workload("cfg2", ndim=2, n=tuple(n), ppc=ppc, dtype="f32", T_keV=T_keV, n_e=n_e,
                  Z=Z, A=A, steps=500, n_ref=6e25, params=p)
    for k, v in kw.items():
        setattr(wl, k, v)
    return wl


def config3(n=(1024, 1024), ppc=32, ratio=100.0, seed=0, **kw) -> Workload:
    """2D 1024x1024, 32 per cell per species, fp32, T = 3 keV, n_e = 6e25,
    lognormal weights (sigma 0.5), all channels forward + inverse, cap 1,
    FP64 feedback with the temperature field evolved, 2000 steps.  ``ratio`` is
    the electron-to-axion macro-weight ratio; the rate boost makes the
    equilibration visible within the run."""
    p = Params(g_agg_GeV=1e-10, g_ae=1e-13, channels=CH_PRIMAKOFF | CH_COMPTON | CH_BREMS,
               inverse=1, lambda_cap=1.0, boost=1e33, feedback=1, T_mode=2, r_relax=0.1,
               seed=seed, hist_lo_keV=0.1, hist_hi_keV=80.0, hist_nbins=128, hist_log=1)
    wl = Workload("cfg3", ndim=2, n=tuple(n), ppc=ppc, dtype="f32", T_keV=3.0, n_e=6e25,
                  Z=1, A=1.0, lognormal_sigma=0.5, steps=2000, params=p)
    wl.params.w_a = (wl.n_e * wl.V_cell_cm3 / ppc) / ratio
    wl.params.w_gamma_prod = 0.0
    for k, v in kw.items():
        setattr(wl, k, v)
    return wl


def config5(n=(256, 256, 256), ppc=32, seed=0, **kw) -> Workload:
    """3D 256^3, Poisson(32) per cell per species, fp32, T linear 1-5 keV and
    n_e linear 1e24-6e25 cm^-3 along x, all channels forward + inverse with
    FP64 feedback, 200 steps.  Every product (axions of all channels, a->gamma
    photons) weighs w_a, the weight of a photon at n_e = 1e24 cm^-3, so that no
    parent is lighter than one product (a lighter one would convert whole, and
    the low-density end would churn photons and axions every step).  Rate boost
    3e30 puts the mean macro-event counts near 1e-2 (Primakoff), 4e-5
    (Compton-like), 2e-6 (brems) and 3e-2 (a->gamma)."""
    p = Params(g_agg_GeV=1e-10, g_ae=1e-13, channels=CH_PRIMAKOFF | CH_COMPTON | CH_BREMS,
               inverse=1, lambda_cap=1.0, boost=3e30, feedback=1, T_mode=2, seed=seed,
               wa_mul=(1.0, 1.0, 1.0),
               hist_lo_keV=0.1, hist_hi_keV=80.0, hist_nbins=128, hist_log=1)
    wl = Workload("cfg5", ndim=3, n=tuple(n), ppc=ppc, dtype="f32", T_keV=1.0, T_keV_hi=5.0,
                  n_e=1e24, n_e_hi=6e25, n_ref=6e25, Z=1, A=1.0, poisson_ppc=True, steps=200,
                  params=p)
    wl.params.w_a = 1e24 * wl.V_cell_cm3 / ppc
    wl.params.w_gamma_prod = wl.params.w_a
    for k, v in kw.items():
        setattr(wl, k, v)
    return wl


# ---------------------------------------------------------------------------
# Rate-surrogate training box: T ~ U[0.5, 10] keV, log n_e ~ U[ln 1e23, ln 1e26],
# Z in {1, 2}, log(omega/T) ~ U[ln 0.01, ln 100], channel uniform over
# (Primakoff, Compton-like, e-Z brems, e-e brems).
# ---------------------------------------------------------------------------
SURROGATE_BOX = dict(T=(0.5, 10.0), ne=(1e23, 1e26), x=(0.01, 100.0))


def surrogate_samples(n: int, seed: int, box: Optional[Dict] = None):
    b = box or SURROGATE_BOX
    rng = np.random.default_rng([seed, 0x5A77])
    T = rng.uniform(b["T"][0], b["T"][1], n)
    ne = np.exp(rng.uniform(math.log(b["ne"][0]), math.log(b["ne"][1]), n))
    Z = rng.integers(1, 3, n).astype(np.float64)
    x = np.exp(rng.uniform(math.log(b["x"][0]), math.log(b["x"][1]), n))
    ch = rng.integers(0, 4, n).astype(np.int32)
    return T, ne, Z, x, ch
