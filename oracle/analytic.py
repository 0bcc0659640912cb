"""Closed-form spectra and integrated powers (test infrastructure).

These are the analytic expectations the Monte-Carlo operators reproduce in
the mean (Sec. III.A-III.D of the paper):

* Compton-like and bremsstrahlung: the emitted number spectrum is
  ``n_e Gamma_c p_c(E)`` (Sec. II.G-II.H), hence the power spectrum
  ``dQ/dE = E n_e Gamma_c p_c(E)`` integrates to ``Q_c = rho eps_c``.
* Primakoff: ``dQ/domega = omega Gamma(omega) dn_gamma/domega`` with the
  blackbody photon density ``omega^2 / (pi^2 (hbar c)^3 (e^{omega/T} - 1))``.
* App. B: absolute spectrum ``dQ/dE = H_k / (V t_tot dE_k)`` in cgs.

All rates come from the oracle's C implementation; this module only
integrates them (scipy's adaptive quadrature serves as the integration step).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize, special

from . import CELL_DTYPE, gamma_prim, const

KEV_ERG = 1.602176634e-9
HBARC_KEVCM = 1.973269804e-8
ZETA5 = 1.0369277551433699263


def pdf_compton(E, T):
    x = np.asarray(E, dtype=np.float64) / T
    return x ** 4 / np.expm1(x) / (24.0 * ZETA5 * T)


def pdf_brems(E, T, k, theta):
    y = np.asarray(E, dtype=np.float64) / (theta * T)
    return np.exp((k - 1.0) * np.log(y) - y - special.gammaln(k)) / (theta * T)


def dQdE_compton(E, cell, params=None):
    """erg cm^-3 s^-1 keV^-1 (no rate boost)."""
    c = np.asarray(cell, dtype=CELL_DTYPE).reshape(())
    nGamma = c["Q_C"] / (c["meanE_C"] * KEV_ERG)
    return np.asarray(E) * nGamma * pdf_compton(E, c["T"]) * KEV_ERG


def dQdE_brems(E, cell, params):
    c = np.asarray(cell, dtype=CELL_DTYPE).reshape(())
    d = params if isinstance(params, dict) else params.as_dict()
    nGamma = c["Q_B"] / (c["meanE_B"] * KEV_ERG)
    return np.asarray(E) * nGamma * pdf_brems(E, c["T"], d["brems_k"], d["brems_theta"]) * KEV_ERG


def dn_blackbody(om, T):
    """Photon number density per keV, both polarisations [cm^-3 keV^-1]."""
    om = np.asarray(om, dtype=np.float64)
    return om ** 2 / (math.pi ** 2 * HBARC_KEVCM ** 3 * np.expm1(om / T))


def dQdE_primakoff(E, cell, params):
    """erg cm^-3 s^-1 keV^-1 for a blackbody photon bath at the cell temperature,
    evaluated with the oracle's Primakoff rate (boost divided out)."""
    c = np.asarray(cell, dtype=CELL_DTYPE).reshape(())
    d = params if isinstance(params, dict) else params.as_dict()
    boost = d.get("boost", 1.0)
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    G = np.array([gamma_prim(c, params, e) for e in E]) / boost
    return E * G * dn_blackbody(E, c["T"]) * KEV_ERG


def integrate_Q(fn, lo, hi, *args):
    f = lambda e: float(np.atleast_1d(fn(np.array([e]), *args))[0])
    # split at a few characteristic energies for robustness
    pts = [p for p in np.geomspace(max(lo, 1e-6), hi, 12)[1:-1]]
    val, err = integrate.quad(f, lo, hi, points=pts, limit=400, epsabs=0.0, epsrel=1e-10)
    return val


def peak(fn, lo, hi, *args):
    """Location and height of the maximum of a smooth spectrum (Brent)."""
    grid = np.geomspace(lo, hi, 400)
    vals = np.array([float(np.atleast_1d(fn(np.array([e]), *args))[0]) for e in grid])
    i = int(np.argmax(vals))
    a, b = grid[max(i - 1, 0)], grid[min(i + 1, grid.size - 1)]
    res = optimize.minimize_scalar(lambda e: -float(np.atleast_1d(fn(np.array([e]), *args))[0]),
                                   bounds=(a, b), method="bounded",
                                   options={"xatol": 1e-10 * b})
    return float(res.x), float(-res.fun)


def hist_edges(params):
    d = params if isinstance(params, dict) else params.as_dict()
    nb, lo, hi = d["hist_nbins"], d["hist_lo_keV"], d["hist_hi_keV"]
    if d["hist_log"]:
        return lo * (hi / lo) ** (np.arange(nb + 1) / nb)
    return lo + (hi - lo) * np.arange(nb + 1) / nb


def absolute_spectrum(H, params, V_total_cm3, t_total_s):
    """App. B: dQ/dE [erg cm^-3 s^-1 keV^-1] from H_k = sum w E [keV]."""
    e = hist_edges(params)
    dE = np.diff(e)
    return H[: dE.size] / (V_total_cm3 * t_total_s * dE) * KEV_ERG


def binned_expectation(fn, params, *args):
    """Integral of a power spectrum over each histogram bin [erg cm^-3 s^-1]."""
    e = hist_edges(params)
    return np.array([integrate.quad(lambda x: float(np.atleast_1d(fn(np.array([x]), *args))[0]),
                                    e[k], e[k + 1], epsrel=1e-10)[0] for k in range(e.size - 1)])
