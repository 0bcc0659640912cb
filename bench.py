#!/usr/bin/env python
"""Throughput of the axion Monte-Carlo hot path on one MI355X.

Workload: the all-channel plasma of the forward benchmark -- 2D 512x512
cells, 64 electrons + 64 H ions + 64 blackbody photons per cell (fp32 SoA),
T = 3 keV, n_e = 6e25 cm^-3, g_agg = 1e-10 GeV^-1, g_ae = 1e-13 -- run
through the whole per-step operator chain:
  axion push + re-binning, cell state, Primakoff conversion on the photons,
  Compton-like + bremsstrahlung emission on the electrons (FP64 power
  histograms), absorption and a->gamma on the axions, FP64 feedback remap.
The temperature field is held fixed (mode (i) of the paper, its benchmark
mode).

One "update" is one (macroparticle, channel) rate evaluation with its
Poisson/Bernoulli draw: 2 per electron, 1 per photon, 3 per axion present at
the start of the step.  `value` = updates/s over the timed steps with all
inputs resident in HBM.  The integrated emitted power per channel is checked
against the closed-form emissivity (<= 1% is the bar) in the CPU leg.

Prints ONE JSON line.  Only one GPU is supported: --gpus N > 1 exits.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic bytes per unit (what the operator must move, fp32 SoA)
ALG_BYTES = {
    "k_prim_count": ("photon", 16),      # p (12 B) + w (4 B)
    "k_therm_count": ("electron", 4),    # w
    "k_abs_count": ("axion", 32),        # p, w, id, cell read + w written
    "k_feedback": ("electron", 40),      # moments (p, w) + remap (p read/write)
    "k_bin": ("axion", 36),              # x, p read; x, cell written (2D)
}
HBM_PEAK_GBPS = 8000.0
TRAFFIC_SUMMARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "hbm_traffic_step_cfg2_512x512.txt")
BF16_PEAK_TFLOPS = 2500.0           # dense BF16 MFMA
# live multiply-adds of the 8-128-128-128-128-1 network, two FLOP each
MLP_FLOP_PER_EVAL = 2 * (8 * 128 + 3 * 128 * 128 + 128)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cells", type=int, default=512, help="grid side (default 512)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--train-steps", type=int, default=20000)
    ap.add_argument("--no-superposed", action="store_true",
                    help="skip the leg with per-cell superposed thermal emission")
    ap.add_argument("--no-massive", action="store_true",
                    help="skip the leg with axions of finite mass")
    ap.add_argument("--mass-keV", type=float, default=1.0,
                    help="axion mass of the finite-mass leg")
    ap.add_argument("--workload", choices=["plasma2d", "graded3d"], default="plasma2d",
                    help="plasma2d: the 512x512 uniform plasma (default); graded3d: the 256^3 "
                         "graded plasma with Poisson per-cell counts (1.6e9 particles, built "
                         "on the GPU; no oracle legs)")
    return ap.parse_args()


def workload(side):
    from paper_2604_24627_amd import inputs as I
    wl = I.config2(T_keV=3.0, n_e=6e25, Z=1, n=(side, side))
    wl.params.inverse = 1
    wl.params.feedback = 1
    wl.params.T_mode = 0
    return wl


def updates_per_step(sim, n_ax0):
    return 2 * sim.el.n + sim.ph.n + 3 * n_ax0


def stream_copy_gbps(torch, B, nbytes=1 << 30, reps=10):
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    L = B.load()
    s = B.stream_handle()
    for _ in range(2):
        B.check(L.axpic_stream_copy(B.ptr(dst), B.ptr(src), nbytes, s), "copy")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        B.check(L.axpic_stream_copy(B.ptr(dst), B.ptr(src), nbytes, s), "copy")
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(wl_full, budget_s):
    """The FP64 oracle, as it stands, on a patch of the same plasma."""
    import numpy as np
    import oracle as O
    from paper_2604_24627_amd import inputs as I
    side = 48
    wl = workload(side)
    pl = I.make_plasma(wl, 1)
    sim = O.OracleSim(pl, wl.params, prec32=True)
    steps, upd = 0, 0
    t0 = time.perf_counter()
    while True:
        n_ax0 = sim.ax.n
        sim.step()
        upd += 2 * sim.el.n + (sim.ph.n) + 3 * n_ax0
        steps += 1
        if time.perf_counter() - t0 > budget_s and steps >= 3:
            break
    dt = time.perf_counter() - t0
    return dict(value=upd / dt, unit="updates/s", cores=O.num_threads(), kind="oracle",
                sample=f"{side}x{side}-cell patch of the same plasma (64 ppc/species, fp32 inputs "
                       f"in FP64), {steps} full steps, {dt:.1f} s")


def analytic_power(wl):
    """Closed-form emissivities [erg cm^-3 s^-1] of the uniform plasma (oracle)."""
    import numpy as np
    import oracle as O
    from oracle import analytic as A
    grid = dict(wl.grid())
    c = O.cell_state(grid, wl.params, np.array([wl.T_keV]), np.array([wl.n_e]),
                     [np.array([wl.n_e / wl.Z])], [float(wl.Z)], [wl.A])[0]
    QP = A.integrate_Q(A.dQdE_primakoff, 1e-4, 400.0, c, wl.params)
    return dict(P=QP, C=float(c["Q_C"]), B=float(c["Q_B"]))


def main_graded(a):
    """The 256^3 graded plasma (T 1-5 keV and n_e 1e24-6e25 cm^-3 along x, Poisson(32)
    particles per cell and species, fp32, all channels forward + inverse, FP64 feedback
    with the temperature evolved): per-particle and superposed thermal emission."""
    import numpy as np
    import torch
    from paper_2604_24627_amd import inputs as I
    from paper_2604_24627_amd import axpic as B
    from paper_2604_24627_amd.sim import AxpicSim
    import gc
    wl = I.config5()
    out = {}
    # one set of inputs serves both legs (each simulation copies what it needs)
    t = time.perf_counter()
    pl = I.make_plasma_device(wl, 0)
    torch.cuda.synchronize()
    print(f"[bench] graded3d inputs built on the GPU in {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)
    for mode in ("particle", "cells"):
        n_ax = int(0.02 * pl["species"]["electrons"]["n"] * (a.steps + a.warmup + 4))
        sim = AxpicSim(pl, wl.params, axion_capacity=n_ax, thermal=mode,
                       photon_extra=int(0.02 * pl["species"]["photons"]["n"]))
        torch.cuda.empty_cache()
        for _ in range(a.warmup):
            sim.step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        upd = 0
        e0.record()
        for _ in range(a.steps):
            upd += updates_per_step(sim, sim.ax.n)
            sim.step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        L = B.load()
        L.axpic_timing_enable(1)
        sim.step()
        torch.cuda.synchronize()
        kt = B.timing_read()
        L.axpic_timing_enable(0)
        out[mode] = {"value": upd / (ms * 1e-3), "ms_per_step": ms / a.steps,
                     "particles": sim.el.n + sim.ion.n + sim.ph.n, "axions_end": sim.ax.n,
                     "hbm_GB_in_use": round(torch.cuda.memory_allocated() / 1e9, 1),
                     "kernel_ms_per_step": {k: round(v[1], 4) for k, v in sorted(kt.items())}}
        print(f"[bench] graded3d {mode}: {ms / a.steps:.3f} ms/step, {out[mode]['value']:.3e} "
              f"updates/s, axions {sim.ax.n}, photons {sim.ph.n}; kernels (ms/step) "
              f"{out[mode]['kernel_ms_per_step']}", file=sys.stderr, flush=True)
        del sim
        gc.collect()
        torch.cuda.empty_cache()
    line = {"metric": "macro-particle rate+sample updates/s, surrogate vs plain, at <=1% power error",
            "value": out["particle"]["value"], "unit": "updates/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": out["particle"]["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "graded 3D plasma 256^3, Poisson(32) e/H-ion/blackbody-photon "
                                   "per cell (fp32 SoA, built on the GPU), T 1-5 keV, n_e "
                                   "1e24-6e25 cm^-3 along x, all channels forward+inverse, FP64 "
                                   "feedback, T evolved", "rate_mode": "plain"},
            "legs": out}
    print(json.dumps(line), flush=True)


def main():
    a = parse()
    if a.workload == "graded3d" and a.gpus == 1:
        return main_graded(a)
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the multi-GPU "
                          "(x-slab) decomposition is a design note, not implemented"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2604_24627_amd import inputs as I
    from paper_2604_24627_amd import axpic as B
    import profsum
    from paper_2604_24627_amd.sim import AxpicSim

    wl = workload(a.cells)
    t = time.perf_counter()
    pl = I.make_plasma(wl)
    print(f"[bench] inputs built in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    est_ax = int(0.01 * 3 * wl.ncell * wl.ppc * (a.steps * 2 + a.warmup + 8))
    sim = AxpicSim(pl, wl.params, axion_capacity=est_ax)
    del pl
    L = B.load()
    for _ in range(a.warmup):
        sim.step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done, axions={sim.ax.n}", file=sys.stderr, flush=True)

    # ---- timed region: throughput
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    upd = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(a.steps):
        upd += updates_per_step(sim, sim.ax.n)
        sim.step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    value = upd / (ms * 1e-3)
    print(f"[bench] timed {a.steps} steps: {ms:.2f} ms (wall {wall * 1e3:.1f} ms), "
          f"{value:.3e} updates/s", file=sys.stderr, flush=True)

    # ---- per-kernel durations (HIP events on the library's stream)
    L.axpic_timing_enable(1)
    n_units = {"photon": [], "electron": [], "axion": []}
    ksteps = max(3, min(a.steps, 10))
    for _ in range(ksteps):
        n_units["photon"].append(sim.ph.n)
        n_units["electron"].append(sim.el.n)
        n_units["axion"].append(sim.ax.n)
        sim.step()
    torch.cuda.synchronize()
    kt = B.timing_read()
    L.axpic_timing_enable(0)
    per_step = {k: v[1] / ksteps for k, v in kt.items()}
    dom = max((k for k in kt if k in ALG_BYTES), key=lambda k: kt[k][1])
    unit, bpu = ALG_BYTES[dom]
    launches, tot_ms = kt[dom]
    avg_ms = tot_ms / launches
    units = float(np.mean(n_units[unit]))
    achieved = units * bpu / (avg_ms * 1e-3) / 1e9
    copy_bw = stream_copy_gbps(torch, B)
    # HBM bytes per launch of that kernel from the committed FETCH_SIZE / WRITE_SIZE summary
    # of this workload (None when the kernels have changed since it was taken)
    tr = profsum.read_traffic(TRAFFIC_SUMMARY, dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": (tr[0] + tr[1]) if tr else None, "avg_ms": round(avg_ms, 5),
                "units_per_launch": units, "bytes_per_unit": bpu,
                "stream_copy_GBps": round(copy_bw, 1)}

    # ---- power of the plain run
    hist = sim.hist_np()
    steps_total = sim.step_index
    V = wl.ncell * wl.V_cell_cm3
    dtp = wl.dt / wl.omega0

    def q_mc(h, nsteps):
        return {ch: float(h[i].sum()) * 1.602176634e-9 / (V * nsteps * dtp)
                for i, ch in enumerate("PCB")}
    Q_mc = q_mc(hist, steps_total)
    counts = {"axions_end": sim.ax.n, "electrons": sim.el.n, "photons": sim.ph.n}
    del sim
    torch.cuda.empty_cache()

    # ---- the same workload with the thermal channels drawn by per-cell superposition
    # (same law; the update count is the per-particle definition's, so the rates compare)
    sup = None
    if not a.no_superposed:
        pl = I.make_plasma(wl)
        sim3 = AxpicSim(pl, wl.params, axion_capacity=est_ax, thermal="cells")
        del pl
        for _ in range(a.warmup):
            sim3.step()
        torch.cuda.synchronize()
        upd3 = 0
        e0.record()
        for _ in range(a.steps):
            upd3 += updates_per_step(sim3, sim3.ax.n)
            sim3.step()
        e1.record()
        torch.cuda.synchronize()
        ms3 = e0.elapsed_time(e1)
        Q_mc3 = q_mc(sim3.hist_np(), sim3.step_index)
        L.axpic_timing_enable(1)
        for _ in range(3):
            sim3.step()
        torch.cuda.synchronize()
        kt3 = B.timing_read()
        L.axpic_timing_enable(0)
        sup = {"value": upd3 / (ms3 * 1e-3), "unit": "updates/s", "ms_per_step": ms3 / a.steps,
               "speed_vs_plain": round((upd3 / (ms3 * 1e-3)) / value, 4),
               "kernel_ms_per_step": {k: round(v[1] / 3, 5) for k, v in sorted(kt3.items())}}
        print(f"[bench] superposed thermal: {ms3 / a.steps:.3f} ms/step, {sup['value']:.3e} "
              f"updates/s", file=sys.stderr, flush=True)
        del sim3
        torch.cuda.empty_cache()

    # ---- the same workload with axions of finite mass (massive kinematics, thresholds,
    # cut spectra, massive absorption); plain rates
    mas = None
    if not a.no_massive:
        import copy
        wlm = copy.deepcopy(wl)
        wlm.params.m_a_keV = a.mass_keV
        pl = I.make_plasma(wlm)
        sim4 = AxpicSim(pl, wlm.params, axion_capacity=est_ax)
        del pl
        for _ in range(a.warmup):
            sim4.step()
        torch.cuda.synchronize()
        upd4 = 0
        e0.record()
        for _ in range(a.steps):
            upd4 += updates_per_step(sim4, sim4.ax.n)
            sim4.step()
        e1.record()
        torch.cuda.synchronize()
        ms4 = e0.elapsed_time(e1)
        L.axpic_timing_enable(1)
        for _ in range(3):
            sim4.step()
        torch.cuda.synchronize()
        kt4 = B.timing_read()
        L.axpic_timing_enable(0)
        mas = {"value": upd4 / (ms4 * 1e-3), "unit": "updates/s", "ms_per_step": ms4 / a.steps,
               "m_a_keV": a.mass_keV, "speed_vs_plain": round((upd4 / (ms4 * 1e-3)) / value, 4),
               "axions_end": sim4.ax.n,
               "kernel_ms_per_step": {k: round(v[1] / 3, 5) for k, v in sorted(kt4.items())}}
        print(f"[bench] massive axions (m = {a.mass_keV} keV): {ms4 / a.steps:.3f} ms/step, "
              f"{mas['value']:.3e} updates/s", file=sys.stderr, flush=True)
        del sim4
        torch.cuda.empty_cache()

    # ---- surrogate form: trained on the GPU outside the timed region, same workload
    sur = sur_tab = None
    if not a.no_surrogate:
        from paper_2604_24627_amd.surrogate import Surrogate
        S = Surrogate(I.Params())
        torch.cuda.synchronize()
        t = time.perf_counter()
        losses = S.train(n_samples=2_000_000, steps=a.train_steps, batch=4096, lr=2e-3,
                         lr_end=2e-5, seed=1)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t
        print(f"[bench] surrogate trained in {t_train:.1f} s, loss {losses[-1][1] if losses else 0:.3e}",
              file=sys.stderr, flush=True)
        def surrogate_leg(mode):
            pl = I.make_plasma(wl)
            sim2 = AxpicSim(pl, wl.params, axion_capacity=est_ax, surrogate=S,
                            surrogate_mode=mode)
            del pl
            for _ in range(a.warmup):
                sim2.step()
            torch.cuda.synchronize()
            upd2 = 0
            e0.record()
            for _ in range(a.steps):
                upd2 += updates_per_step(sim2, sim2.ax.n)
                sim2.step()
            e1.record()
            torch.cuda.synchronize()
            ms2 = e0.elapsed_time(e1)
            res = {"value": upd2 / (ms2 * 1e-3), "unit": "updates/s",
                   "ms_per_step": ms2 / a.steps, "train_s": round(t_train, 2),
                   "train_steps": a.train_steps, "train_samples": 2_000_000,
                   "final_loss": losses[-1][1] if losses else None,
                   "fallback_evals": int(sim2.fallback.item()),
                   "speed_vs_plain": round((upd2 / (ms2 * 1e-3)) / value, 4)}
            Q = q_mc(sim2.hist_np(), sim2.step_index)
            print(f"[bench] surrogate ({mode}): {ms2 / a.steps:.3f} ms/step, "
                  f"{res['value']:.3e} updates/s", file=sys.stderr, flush=True)
            # the network kernel against the matrix-core peak.  Evaluations per step:
            # per particle, photons (lambda_P) + 4 per old axion (three thermal channels and
            # a->gamma); per cell, nodes x (Primakoff + three thermal channels)
            L.axpic_timing_enable(1)
            evals = 0
            for _ in range(3):
                if mode == "particle":
                    evals += sim2.ph.n + 4 * sim2.ax.n
                else:
                    evals += sim2.ncell * S.TABLE_NODES * 4
                sim2.step()
            torch.cuda.synchronize()
            kt2 = B.timing_read()
            L.axpic_timing_enable(0)
            kname = "k_rates_mlp" if mode == "particle" else "k_mlp_table"
            if kname in kt2:
                launches2, tot2 = kt2[kname]
                tflops = evals * MLP_FLOP_PER_EVAL / (tot2 * 1e-3) / 1e12
                res["roofline"] = {"bound": "mfma", "kernel": kname,
                                   "achieved": round(tflops, 1), "peak": BF16_PEAK_TFLOPS,
                                   "unit": "TFLOP/s", "frac": round(tflops / BF16_PEAK_TFLOPS, 4),
                                   "traffic": None, "avg_ms": round(tot2 / launches2, 5),
                                   "evals_per_step": evals / 3,
                                   "flop_per_eval": MLP_FLOP_PER_EVAL}
            if mode == "table":
                res["table"] = {"nodes": S.TABLE_NODES, "x_range": list(S.TABLE_RANGE)}
            res["kernel_ms_per_step"] = {k: round(v[1] / 3, 5) for k, v in sorted(kt2.items())}
            del sim2
            torch.cuda.empty_cache()
            return res, Q
        sur, Q_mc2 = surrogate_leg("particle")
        sur_tab, Q_mc4 = surrogate_leg("table")

    # ---- power check against the closed-form emissivities, CPU baseline (oracle)
    power = None
    cpu = None
    if not a.no_cpu_baseline:
        Qa = analytic_power(wl)
        power = {ch: round(Q_mc[ch] / Qa[ch] - 1.0, 5) for ch in "PCB"}
        if sur is not None:
            sur["power_err"] = {ch: round(Q_mc2[ch] / Qa[ch] - 1.0, 5) for ch in "PCB"}
            sur_tab["power_err"] = {ch: round(Q_mc4[ch] / Qa[ch] - 1.0, 5) for ch in "PCB"}
        if sup is not None:
            sup["power_err"] = {ch: round(Q_mc3[ch] / Qa[ch] - 1.0, 5) for ch in "PCB"}
        cpu = cpu_baseline(wl, a.cpu_seconds)

    out = {
        "metric": "macro-particle rate+sample updates/s, surrogate vs plain, at <=1% power error",
        "value": value, "unit": "updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms / a.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"uniform thermal plasma, 2D {a.cells}x{a.cells} cells, 64 "
                               "e/H-ion/blackbody-photon per cell (fp32 SoA), T=3 keV, "
                               "n_e=6e25 cm^-3, all channels forward+inverse, FP64 feedback, "
                               "T fixed", "rate_mode": "plain",
                   **counts},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "power_err": power,
        "kernel_ms_per_step": {k: round(v, 5) for k, v in sorted(per_step.items())},
        "surrogate": sur,
        "surrogate_table": sur_tab,
        "superposed_thermal": sup,
        "massive_axions": mas,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
