"""Per-cell tables of the rate surrogate and their per-particle interpolation,
in FP64 (test infrastructure: the reference the table entry points of the
library are checked against; nothing outside tests/ uses it).

Reading.  Apart from omega, every input of the surrogate -- T, kappa (eq.
kappa_debye), n_e and Z -- is a property of the cell (Sec. II.E), so for one
cell the learned log-rate is a function of u = ln(omega/T) alone.  It is
evaluated at the nodes u_j = ln x_lo + j h, h = (ln x_hi - ln x_lo)/(nodes - 1),
and a particle takes the cubic through the four nodes around it.

Slots of a cell's table:
  0  log R_P, R_P = Gamma_{gamma->a}/g_agg^2 as the network predicts it;
  1  log sum_c f_c R_c over the enabled thermal channels c (Compton-like,
     e-Z brems, e-e brems if brems_ee): R_c = Gamma_abs,c/g_ae^2 (eq.
     gamma_abs) as predicted, f_c = 1 for Compton and the screening-fit
     factor max(0, 1 - a eta) of eqs. eps_eZ / eps_ee for brems (a = 6.98e-2
     e-Z, 0.140 e-e; eta = (3 + X_H) rho_2 / T_7^2).
A cell outside the training box (T, n_e, one ion species of charge 1 or 2)
has NaN entries; its particles use the plain rate.
"""
from __future__ import annotations

import math

import numpy as np

from . import mlp as M

KEV_T7 = 1.160451812         # T_7 = T[keV] * this (1 keV = 1.160451812e7 K)
A_SCREEN = (6.98e-2, 0.140)  # screening-fit slopes of eqs. eps_eZ, eps_ee


def grid(x_lo: float, x_hi: float, nodes: int):
    """(u0, h) of the node grid u_j = u0 + j h over [ln x_lo, ln x_hi]."""
    u0 = math.log(x_lo)
    return u0, (math.log(x_hi) - u0) / (nodes - 1)


def interpolate(values, u0: float, h: float, u):
    """The cubic through the four nodes around each u, in Lagrange form.

    values: [n, nodes] node values per particle (or [nodes] for all); u: [n].
    The stencil starts at k = clamp(floor(t) - 1, 0, nodes - 4), t = (u - u0)/h,
    so an interior point sits between the stencil's middle nodes and the end
    intervals use the first or last four nodes."""
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    V = np.asarray(values, dtype=np.float64)
    if V.ndim == 1:
        V = np.broadcast_to(V, (u.size, V.size))
    nodes = V.shape[1]
    t = (u - u0) / h
    k = np.clip(np.floor(t).astype(np.int64) - 1, 0, nodes - 4)
    out = np.zeros(u.size)
    rows = np.arange(u.size)
    for m in range(4):
        basis = np.ones(u.size)
        for q in range(4):
            if q != m:
                basis *= (t - (k + q)) / (m - q)
        out += basis * V[rows, k + m]
    return out


def screening_factor(T_keV, rho, XH, ee: bool):
    """max(0, 1 - a eta), eta = (3 + X_H)(rho/100)/T_7^2 (eqs. eps_eZ, eps_ee)."""
    T7 = np.asarray(T_keV, dtype=np.float64) * KEV_T7
    eta = (3.0 + np.asarray(XH)) * (np.asarray(rho) / 100.0) / (T7 * T7)
    return np.maximum(0.0, 1.0 - A_SCREEN[1 if ee else 0] * eta)


def log_rate(P, norm, feat, ch, quantize=True):
    """The surrogate's log R for raw features feat [n, 4] = (ln x, ln(kappa/T),
    ln n_e, Z) and channel ch: mu_ch + lin_ch . f + sigma_ch y(f, onehot_ch) with
    the normalised f_i = (feat_i - lo_i) sc_i - 1."""
    feat = np.asarray(feat, dtype=np.float64)
    f = (feat - np.asarray(norm["feat_lo"])) * np.asarray(norm["feat_sc"]) - 1.0
    onehot = np.zeros((feat.shape[0], 4))
    onehot[:, ch] = 1.0
    y, _ = M.forward(P, np.concatenate([f, onehot], axis=1), quantize=quantize)
    lin = np.asarray(norm["out_lin"], dtype=np.float64).reshape(4, 4)[ch]
    return norm["out_mu"][ch] + f @ lin + norm["out_sigma"][ch] * y


def cell_tables(P, norm, box, cells, Z, nion, params, nodes, x_range=None, quantize=True):
    """Tables [ncell, 2, nodes] for the oracle's cell records `cells` (fields T,
    n_e, kappa2, rho, XH), ion charge Z of a single ion species (nion = 1), on
    nodes over x_range (default: the training range box["x"])."""
    T = np.asarray(cells["T"], dtype=np.float64)
    ne = np.asarray(cells["n_e"], dtype=np.float64)
    ncell = T.size
    x_lo, x_hi = box["x"] if x_range is None else x_range
    u0, h = grid(x_lo, x_hi, nodes)
    u = u0 + h * np.arange(nodes)
    feat = np.empty((ncell, nodes, 4))
    feat[:, :, 0] = u[None, :]
    feat[:, :, 1] = (0.5 * np.log(cells["kappa2"]) - np.log(T))[:, None]
    feat[:, :, 2] = np.log(ne)[:, None]
    feat[:, :, 3] = Z
    feat = feat.reshape(-1, 4)
    out = np.empty((ncell, 2, nodes))
    out[:, 0, :] = log_rate(P, norm, feat, 0, quantize).reshape(ncell, nodes)
    on = [(params["channels"] & 2) != 0, (params["channels"] & 4) != 0,
          (params["channels"] & 4) != 0 and bool(params["brems_ee"])]
    total = np.zeros((ncell, nodes))
    for ch in (1, 2, 3):
        if not on[ch - 1]:
            continue
        f = 1.0 if ch == 1 else screening_factor(T, cells["rho"], cells["XH"], ch == 3)[:, None]
        total += f * np.exp(log_rate(P, norm, feat, ch, quantize).reshape(ncell, nodes))
    with np.errstate(divide="ignore"):
        out[:, 1, :] = np.log(total)
    inside = ((nion == 1) & (Z in (1.0, 2.0)) & (T >= box["T"][0]) & (T <= box["T"][1]) &
              (ne >= box["ne"][0]) & (ne <= box["ne"][1]))
    out[~inside] = np.nan
    return out


def table_rates(tables, x_range, mode, T_cell, cell, omega_keV, w, params, dt_phys, units):
    """Per-particle rates from tables [ncell, 2, nodes] on nodes over x_range.

    mode 0 (photons): lambda = w units["P"] (1 - exp(-g_agg^2 B R_P dt));
    mode 2 (axions, a->gamma): lambda = w units["ag"] (1 - exp(-r g_agg^2 B R_P dt));
    mode 1 (axions): P_abs = 1 - exp(-g_ae^2 B R_abs dt)  (eq. gamma_abs summed
    over the thermal channels; zero if that sum is zero).
    B = params' boost, r = prim_inv_ratio; w <= 0 gives 0.  Returns (rates,
    use_table): particles outside x_range or in a NaN cell have
    use_table False and rate NaN (the caller's plain rate applies there)."""
    tables = np.asarray(tables, dtype=np.float64)
    nodes = tables.shape[2]
    x_lo, x_hi = x_range
    u0, h = grid(x_lo, x_hi, nodes)
    x = np.asarray(omega_keV, dtype=np.float64) / np.asarray(T_cell)[cell]
    slot = tables[cell, 1 if mode == 1 else 0, :]
    use = ~np.isnan(slot[:, 0]) & (x >= x_lo) & (x <= x_hi)
    rate = np.full(x.size, np.nan)
    idx = np.nonzero(use)[0]
    if idx.size:
        sl = slot[idx]
        zero = np.isneginf(sl[:, 0])
        L = interpolate(np.where(zero[:, None], 0.0, sl), u0, h, np.log(x[idx]))
        R = np.where(zero, 0.0, np.exp(L))
        B = params["boost"]
        if mode == 0:
            r = np.asarray(w)[idx] * units["P"] * -np.expm1(-params["g_agg_GeV"] ** 2 * B * R * dt_phys)
        elif mode == 2:
            r = np.asarray(w)[idx] * units["ag"] * -np.expm1(
                -params["prim_inv_ratio"] * params["g_agg_GeV"] ** 2 * B * R * dt_phys)
        else:
            r = -np.expm1(-params["g_ae"] ** 2 * B * R * dt_phys)
        r[~(np.asarray(w)[idx] > 0)] = 0.0
        rate[idx] = r
    return rate, use


def particle_rates(P, norm, box, cells, Z, nion, params, mode, cell, omega_keV, w, dt_phys,
                   units, quantize=True):
    """Per-particle rates of the surrogate without tables, in FP64 (the reference of the
    library's per-particle inference): for each particle the features come from its
    energy omega and its cell's record (T, kappa2, n_e; Z of the single ion species),
    log R from the network, and

    mode 0 (photons):        lambda = w units["P"] (1 - exp(-g_agg^2 B R_P dt));
    mode 2 (axions, a->g):   lambda = w units["ag"] (1 - exp(-r g_agg^2 B R_P dt));
    mode 1 (axions):         P_abs = 1 - exp(-g_ae^2 B sum_c f_c R_c dt) over the enabled
                             thermal channels (f_c as in the tables' slot 1),
    B the boost, r = prim_inv_ratio; w <= 0 gives 0.  Returns (rates, inside): a
    particle whose cell lies outside the training box (T, n_e, one ion species of
    charge 1 or 2) or whose omega/T lies outside box["x"] has inside False and rate
    NaN (the caller's plain rate applies there)."""
    cell = np.asarray(cell, dtype=np.int64)
    T = np.asarray(cells["T"], dtype=np.float64)[cell]
    ne = np.asarray(cells["n_e"], dtype=np.float64)[cell]
    k2 = np.asarray(cells["kappa2"], dtype=np.float64)[cell]
    om = np.asarray(omega_keV, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    x = om / T
    inside = ((nion == 1) & (Z in (1.0, 2.0)) & (T >= box["T"][0]) & (T <= box["T"][1]) &
              (ne >= box["ne"][0]) & (ne <= box["ne"][1]) & (x >= box["x"][0]) &
              (x <= box["x"][1]))
    rate = np.full(om.size, np.nan)
    idx = np.nonzero(inside)[0]
    if idx.size == 0:
        return rate, inside
    with np.errstate(divide="ignore"):
        feat = np.stack([np.log(x[idx]), 0.5 * np.log(k2[idx]) - np.log(T[idx]), np.log(ne[idx]),
                         np.full(idx.size, float(Z))], axis=1)
    B = params["boost"]
    if mode in (0, 2):
        R = np.exp(log_rate(P, norm, feat, 0, quantize))
        G = params["g_agg_GeV"] ** 2 * B * R * dt_phys
        if mode == 0:
            r = w[idx] * units["P"] * -np.expm1(-G)
        else:
            r = w[idx] * units["ag"] * -np.expm1(-params["prim_inv_ratio"] * G)
    else:
        on = [(params["channels"] & 2) != 0, (params["channels"] & 4) != 0,
              (params["channels"] & 4) != 0 and bool(params["brems_ee"])]
        rho = np.asarray(cells["rho"], dtype=np.float64)[cell][idx]
        XH = np.asarray(cells["XH"], dtype=np.float64)[cell][idx]
        tot = np.zeros(idx.size)
        for ch in (1, 2, 3):
            if not on[ch - 1]:
                continue
            f = 1.0 if ch == 1 else screening_factor(T[idx], rho, XH, ch == 3)
            tot += f * np.exp(log_rate(P, norm, feat, ch, quantize))
        r = -np.expm1(-params["g_ae"] ** 2 * B * tot * dt_phys)
    r[~(w[idx] > 0)] = 0.0
    rate[idx] = r
    return rate, inside
