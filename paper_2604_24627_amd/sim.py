"""Host driver of one time step of the axion Monte-Carlo operators on one GPU.

Buffers are torch tensors on the device (memory and streams only); every
operator is a call into libaxpic.so.  The step order is the one the operators
are defined with: every operator acts on the population present at the start
of the step, and the feedback is applied last:

  1. push the axions present at the start of the step, re-bin them and put them in
     the canonical order (stable by cell, zero weights dropped);
  2. local state of every cell (deposits, temperature field -> prefactors);
  3. forward Primakoff on the photons; thermal emission on the electrons;
  4. absorption and a->gamma on the axions present before step 3;
  5. feedback remap of the electrons and temperature update.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional

import numpy as np
import torch

from . import axpic as B


def _tdtype(dt: int):
    return torch.float32 if dt == B.F32 else torch.float64


class DeviceSpecies:
    """SoA macroparticle buffer on the GPU with host-side length/capacity."""

    def __init__(self, kind: int, dtype: int, ndim: int, capacity: int, w_ref: float,
                 device, Z: float = 0.0, A: float = 0.0, with_p: bool = True,
                 cache_p2: bool = True):
        self.kind, self.dtype, self.ndim = kind, dtype, ndim
        self.w_ref, self.Z, self.A = float(w_ref), float(Z), float(A)
        self.device = device
        self.with_p = with_p
        # photons keep |p|^2 beside p: their conversion rate needs only that
        self.with_p2 = with_p and kind == B.PHOTON and cache_p2
        self.p2 = None
        self.n = 0
        self.capacity = 0
        self.x = [None, None, None]
        self.p = [None, None, None]
        self.w = self.id = self.cell = None
        self.off = None         # per-cell offsets of the cell-ordered prefix [0, n_sorted)
        self.n_sorted = 0
        self.id0 = 0
        self.n_implicit = 0
        self.grows = 0          # reallocations after the first (each copies the buffers)
        self._alloc(max(int(capacity), 1))

    def _alloc(self, cap: int):
        td = _tdtype(self.dtype)
        dev = self.device
        self._S = None          # the cached C view points at the buffers being replaced

        def grow(t, dt_):
            # no kernel reads a slot at or beyond n before writing it: no fill needed
            new = torch.empty(cap, dtype=dt_, device=dev)
            if t is not None and self.n:
                new[: self.n].copy_(t[: self.n])
            return new
        for d in range(3):
            self.x[d] = grow(self.x[d], td) if d < self.ndim else None
            self.p[d] = grow(self.p[d], td) if self.with_p else None
        self.p2 = grow(self.p2, td) if self.with_p2 else None
        self.w = grow(self.w, td)
        self.id = grow(self.id, torch.int64)
        self.cell = grow(self.cell, torch.int32)
        self.grows += 1 if self.capacity else 0
        self.capacity = cap

    def ensure(self, cap: int):
        """Room for cap particles; grows geometrically, by half at least (each growth
        copies the buffers)."""
        if cap > self.capacity:
            self._alloc(max(int(cap * 1.25), int(1.5 * self.capacity)) + 1024)

    @staticmethod
    def from_input(sp: Dict, kind: int, ndim: int, device, extra: int = 0) -> "DeviceSpecies":
        if isinstance(sp["w"], torch.Tensor):
            return DeviceSpecies._from_device(sp, kind, ndim, device, extra)
        dt = B.F64 if sp["w"].dtype == np.float64 else B.F32
        n = int(sp["n"])
        s = DeviceSpecies(kind, dt, ndim, n + extra, sp["w_ref"], device, sp["Z"], sp["A"],
                          with_p=sp["p"] is not None)
        s.n = n
        for d in range(ndim):
            s.x[d][:n].copy_(torch.from_numpy(np.ascontiguousarray(sp["x"][d])))
        if sp["p"] is not None:
            for d in range(3):
                s.p[d][:n].copy_(torch.from_numpy(np.ascontiguousarray(sp["p"][d])))
        s.w[:n].copy_(torch.from_numpy(sp["w"]))
        s.id[:n].copy_(torch.from_numpy(sp["id"].view(np.int64)))
        s.cell[:n].copy_(torch.from_numpy(sp["cell"]))
        s.off = torch.from_numpy(sp["off"]).to(device)
        s.n_sorted = n
        ids = sp["id"]
        if n and np.array_equal(ids, ids[0] + np.arange(n, dtype=np.uint64)):
            s.id0, s.n_implicit = int(ids[0]), n
        return s

    @staticmethod
    def _from_device(sp: Dict, kind: int, ndim: int, device, extra: int) -> "DeviceSpecies":
        """From device tensors (inputs.make_plasma_device); ids implicit from id0."""
        dt = B.F64 if sp["w"].dtype == torch.float64 else B.F32
        n = int(sp["n"])
        s = DeviceSpecies(kind, dt, ndim, n + extra, sp["w_ref"], device, sp["Z"], sp["A"],
                          with_p=sp["p"] is not None)
        s.n = n
        for d in range(ndim):
            s.x[d][:n].copy_(sp["x"][d])
        if sp["p"] is not None:
            for d in range(3):
                s.p[d][:n].copy_(sp["p"][d])
        s.w[:n].copy_(sp["w"])
        torch.arange(sp["id0"], sp["id0"] + n, out=s.id[:n])
        s.cell[:n].copy_(sp["cell"])
        s.off = sp["off"].to(device)
        s.n_sorted = n
        s.id0, s.n_implicit = int(sp["id0"]), n
        return s

    def struct(self) -> B.SpeciesC:
        """The C view of the buffer (cached while the buffers, offsets and implicit-id
        range stay the same; n is refreshed on every call)."""
        key = (id(self.off), self.n_sorted, self.id0, self.n_implicit, self.w_ref)
        S = getattr(self, "_S", None)
        if S is None or self._S_key != key:
            S = B.SpeciesC()
            for d in range(3):
                S.x[d] = B.ptr(self.x[d])
                S.p[d] = B.ptr(self.p[d])
            S.w, S.id, S.cell = B.ptr(self.w), B.ptr(self.id), B.ptr(self.cell)
            S.p2 = B.ptr(self.p2) if self.p2 is not None else None
            S.dtype, S.kind = self.dtype, self.kind
            S.w_ref, S.Z, S.A = self.w_ref, self.Z, self.A
            S.id0, S.n_implicit = self.id0, self.n_implicit
            S.off, S.n_sorted = ((B.ptr(self.off), self.n_sorted) if self.off is not None
                                 else (None, 0))
            self._S, self._S_key = S, key
        S.n, S.capacity = self.n, self.capacity
        return S

    def fill_p2(self, lib, stream, start: int = 0):
        """|p|^2 of particles start .. n-1 from their momenta (the photons' cache)."""
        if self.p2 is not None:
            B.check(lib.axpic_fill_p2(B.ref(self.struct()), int(start), stream), "fill_p2")

    def to_numpy(self) -> Dict:
        n = self.n
        out = dict(w=self.w[:n].cpu().numpy(), id=self.id[:n].cpu().numpy().view(np.uint64),
                   cell=self.cell[:n].cpu().numpy())
        out["x"] = np.stack([self.x[d][:n].cpu().numpy() if self.x[d] is not None
                             else np.zeros(n, dtype=out["w"].dtype) for d in range(3)])
        out["p"] = (np.stack([self.p[d][:n].cpu().numpy() for d in range(3)])
                    if self.with_p else None)
        return out


class AxpicSim:
    """One uniform-grid run on the current GPU."""

    def __init__(self, plasma: Dict, params, device: str = "cuda", axion_capacity: int = 0,
                 photon_extra: int = 0, compact_every: int = 0, stream=None, surrogate=None,
                 thermal: str = "particle", surrogate_mode: str = "particle", sort: bool = True):
        self.lib = B.load()
        self._allocs = 0            # workspaces and spare buffers made (see reallocations)
        self.device = torch.device(device)
        self.pdict = dict(params if isinstance(params, dict) else params.as_dict())
        self.params = B.make_params(self.pdict)
        self.grid_d = plasma["grid"]
        self.grid = B.make_grid(self.grid_d)
        self.ndim = self.grid_d["ndim"]
        sp = plasma["species"]
        self.el = DeviceSpecies.from_input(sp["electrons"], B.ELECTRON, self.ndim, self.device)
        self.ion = DeviceSpecies.from_input(sp["ions"], B.ION, self.ndim, self.device)
        self.ph = DeviceSpecies.from_input(sp["photons"], B.PHOTON, self.ndim, self.device,
                                           extra=photon_extra)
        self.dtype = self.el.dtype
        cap = axion_capacity or max(4096, self.ph.n // 8)
        self.ax = DeviceSpecies(B.AXION, self.dtype, self.ndim, cap, self.pdict["w_a"], self.device)
        self.ncell = int(np.prod(self.grid_d["n"]))
        self.next_id = int(plasma["next_id"])
        self.compact_every = compact_every
        self.step_index = 0
        dev = self.device
        f64 = torch.float64
        self.T = torch.from_numpy(plasma["T_cell"]).to(dev, f64).clone()
        self.dens = torch.zeros((1 + B.MAX_IONS) * self.ncell, dtype=f64, device=dev)
        self.state = torch.zeros(self.ncell * B.STATE_N, dtype=f64, device=dev)
        self.pref32 = torch.zeros(self.ncell * B.PREF_N, dtype=torch.float32, device=dev)
        self.pref64 = torch.zeros(self.ncell * B.PREF_N, dtype=f64, device=dev)
        self.cells = B.CellsC()
        self.cells.ncell = self.ncell
        self.cells.T_keV, self.cells.dens = B.ptr(self.T), B.ptr(self.dens)
        self.cells.state, self.cells.pref32, self.cells.pref64 = (B.ptr(self.state),
                                                                  B.ptr(self.pref32),
                                                                  B.ptr(self.pref64))
        self.cells.nion = 1
        self.cells.Zion[0], self.cells.Aion[0] = self.ion.Z, self.ion.A
        nb = self.pdict["hist_nbins"] + 2
        self.hist = torch.zeros(3 * nb, dtype=f64, device=dev)
        self.stats = torch.zeros(B.ST_COUNT, dtype=f64, device=dev)
        self.fb = torch.zeros(self.ncell * 4, dtype=f64, device=dev)
        self.status = torch.zeros(B.STATUS_N, dtype=torch.int64, device=dev)
        self.diag_out = torch.zeros(2, dtype=f64, device=dev)
        self.ws = None
        self.ws_bytes = 0
        self._ensure_ws(max(self.el.n, self.ph.n, self.ax.capacity, 2 * self.ncell))
        self.stream = stream
        s = self.sh
        self.ph.fill_p2(self.lib, s)
        B.check(self.lib.axpic_deposit(B.ref(self.grid), B.ref(self.el.struct()), B.ptr(self.el.off),
                                       B.ref(self.cells), 0, s), "deposit electrons")
        B.check(self.lib.axpic_deposit(B.ref(self.grid), B.ref(self.ion.struct()),
                                       B.ptr(self.ion.off), B.ref(self.cells), 1, s),
                "deposit ions")
        self.cell_state()
        self.need_feedback = bool(self.pdict["feedback"] or self.pdict["T_mode"] == 2)
        # learned rate backend for the per-particle, energy-dependent rates (photon conversion,
        # axion absorption and a->gamma); None = plain closed forms
        self.surrogate = surrogate
        # "particle": one network pass per particle (axpic_rates_mlp); "table": per-cell
        # tables on a grid of omega/T, interpolated per particle (axpic_mlp_table,
        # axpic_rates_table)
        if surrogate_mode not in ("particle", "table"):
            raise ValueError(surrogate_mode)
        self.surrogate_mode = surrogate_mode
        self._tab = None
        self.fallback = torch.zeros(1, dtype=torch.int64, device=self.device)
        # device chain of the step's appending calls {axions, photons, next id, skip} and
        # one status record per call
        self.chain = torch.zeros(B.CHAIN_N, dtype=torch.int64, device=dev)
        self.chain_host = torch.zeros(B.CHAIN_N, dtype=torch.int64).pin_memory()
        self._chain_np = self.chain_host.numpy()
        self.status_ops = torch.zeros((3, B.STATUS_N), dtype=torch.int64, device=dev)
        self._last_new = (0, 0)
        self.grow_ahead = True      # reserve room for twice the previous step's products
        self._spare = {}            # compaction targets by kind, reused
        # canonical order of the axions after every push (axpic_sort_cells): stable by
        # cell, zero weights dropped, cell offsets kept for the operators
        self.sort = sort
        # the surrogate's axion rates need the kept count on the host before the calls, so
        # its steps sort unchained (a read-back); the plain steps chain the sort
        self.sort_chained = surrogate is None
        self.ax_off = torch.zeros(self.ncell + 1, dtype=torch.int64, device=dev)
        self.sort_status = torch.zeros(B.STATUS_N, dtype=torch.int64, device=dev)
        self.sort_ws = None
        # thermal emission: "particle" (a Poisson draw per electron and channel) or
        # "cells" (per-cell superposition, axpic_sample_emit_cells)
        if thermal not in ("particle", "cells"):
            raise ValueError(thermal)
        self.thermal = thermal
        self.cellw = None
        if thermal == "cells":
            self.cellw = torch.zeros(2 * self.ncell, dtype=f64, device=dev)
            B.check(self.lib.axpic_cell_weights(B.ref(self.el.struct()), B.ptr(self.el.off),
                                                self.ncell, B.ptr(self.cellw), s), "cell_weights")
            self._ensure_ws(4 * self.ncell)

    def load_axions(self, sp: Dict, extra: int = 0):
        """Replace the axion buffer by a given population (a make_plasma-style species
        dict of relative weights with w_ref = w_a); ids after it are issued from its
        next_id on."""
        if abs(sp["w_ref"] - self.pdict["w_a"]) > 1e-12 * abs(self.pdict["w_a"]):
            raise ValueError("axion w_ref must equal the parameters' w_a")
        ax = DeviceSpecies.from_input(sp, B.AXION, self.ndim, self.device, extra=extra)
        if ax.dtype != self.dtype:
            raise ValueError("axion dtype differs from the plasma's")
        ax.id0 = ax.n_implicit = 0          # every id stored: appended ids continue elsewhere
        ax.off, ax.n_sorted = None, 0       # axions move: no cell-ordered prefix
        self.ax = ax
        self.next_id = max(self.next_id, int(sp.get("next_id", 0)))
        self._ensure_ws(self.ax.capacity)

    @property
    def sh(self):
        return B.stream_handle(self.stream)

    def _ensure_ws(self, n: int):
        need = self.lib.axpic_workspace_bytes(int(n))
        if need > self.ws_bytes:
            need = int(need * 1.25) + 4096
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self.ws_bytes = need
            self._allocs += 1

    def reallocations(self) -> int:
        """Device buffers (re)allocated so far after set-up: particle buffers grown, spare
        buffers and workspaces made or enlarged (a step without any allocates nothing)."""
        sp = [self.el, self.ion, self.ph, self.ax] + list(self._spare.values())
        return self._allocs + sum(s.grows for s in sp)

    # -------------------------------------------------------------- checkpoint
    _CKPT_SPECIES = ("el", "ion", "ph", "ax")

    def save(self, path: str):
        """Write what the following steps depend on to the directory `path`: the four
        particle buffers (their first n particles, the offsets of a cell-ordered prefix,
        the implicit-id range), the cell temperatures, the accumulated statistics and
        histograms, the step index and the next id.  There is no random state to keep:
        every draw is keyed by (seed, particle id, step).  The cell state and the
        prefactors are derived from the temperatures on load; workspaces, spare buffers
        and the device chain are scratch.  A surrogate is not saved: the caller hands
        the same one to the sim it loads into."""
        from safetensors.torch import save_file
        os.makedirs(path, exist_ok=True)
        t = {"T": self.T, "stats": self.stats, "hist": self.hist}
        meta = {"step_index": self.step_index, "next_id": self.next_id,
                "last_new": list(self._last_new), "ncell": self.ncell, "species": {}}
        for name in self._CKPT_SPECIES:
            sp = getattr(self, name)
            n = sp.n
            for d in range(3):
                if sp.x[d] is not None:
                    t[f"{name}.x{d}"] = sp.x[d][:n]
                if sp.p[d] is not None:
                    t[f"{name}.p{d}"] = sp.p[d][:n]
            t[f"{name}.w"], t[f"{name}.id"], t[f"{name}.cell"] = sp.w[:n], sp.id[:n], sp.cell[:n]
            if sp.off is not None:
                t[f"{name}.off"] = sp.off
            meta["species"][name] = {"n": n, "n_sorted": sp.n_sorted, "id0": sp.id0,
                                     "n_implicit": sp.n_implicit, "w_ref": sp.w_ref,
                                     "dtype": sp.dtype, "has_off": sp.off is not None}
        save_file({k: v.detach().contiguous().cpu() for k, v in t.items()},
                  os.path.join(path, "state.safetensors"))
        with open(os.path.join(path, "state.json"), "w") as f:
            json.dump(meta, f)

    def load(self, path: str):
        """Continue from a checkpoint written by save() of a sim built from the same
        plasma and parameters: the following steps then equal, bit for bit, those of the
        sim that wrote it."""
        from safetensors.torch import load_file
        with open(os.path.join(path, "state.json")) as f:
            meta = json.load(f)
        if meta["ncell"] != self.ncell:
            raise ValueError("checkpoint of a different grid")
        t = load_file(os.path.join(path, "state.safetensors"), device=str(self.device))
        for name in self._CKPT_SPECIES:
            sp = getattr(self, name)
            m = meta["species"][name]
            if m["dtype"] != sp.dtype or m["w_ref"] != sp.w_ref:
                raise ValueError(f"checkpoint {name}: dtype or reference weight differs")
            n = int(m["n"])
            sp.ensure(n)
            sp.n = n
            for d in range(3):
                if sp.x[d] is not None:
                    sp.x[d][:n].copy_(t[f"{name}.x{d}"])
                if sp.p[d] is not None:
                    sp.p[d][:n].copy_(t[f"{name}.p{d}"])
            sp.w[:n].copy_(t[f"{name}.w"])
            sp.id[:n].copy_(t[f"{name}.id"])
            sp.cell[:n].copy_(t[f"{name}.cell"])
            sp.id0, sp.n_implicit, sp.n_sorted = int(m["id0"]), int(m["n_implicit"]), int(m["n_sorted"])
            if not m["has_off"]:
                sp.off = None
            elif name == "ax":
                self.ax_off.copy_(t["ax.off"])
                sp.off = self.ax_off
            else:
                sp.off = t[f"{name}.off"].clone()
            sp._S = None
        self.T.copy_(t["T"])
        self.stats.copy_(t["stats"])
        self.hist.copy_(t["hist"])
        self.step_index, self.next_id = int(meta["step_index"]), int(meta["next_id"])
        self._last_new = tuple(meta["last_new"])
        self._ensure_ws(max(self.el.n, self.ph.n, self.ax.capacity, 2 * self.ncell))
        self.ph.fill_p2(self.lib, self.sh)
        self.cell_state()
        if self.cellw is not None:
            B.check(self.lib.axpic_cell_weights(B.ref(self.el.struct()), B.ptr(self.el.off),
                                                self.ncell, B.ptr(self.cellw), self.sh),
                    "cell_weights")

    def domain_cells(self) -> int:
        """Cells whose temperature or a density lies outside the model's domain (negative
        or not finite) at the last cell-state pass; nothing is emitted or absorbed there."""
        return int((self.state.view(-1, B.STATE_N)[:, B.STATE_N - 1] != 0.0).sum())

    def cell_state(self):
        B.check(self.lib.axpic_cell_state(B.ref(self.grid), B.ref(self.cells), B.ref(self.params),
                                          self.el.w_ref, self.ph.w_ref, self.sh), "cell_state")

    # -------------------------------------------------------------- operators
    def _append_call(self, fn, out_species: DeviceSpecies, what: str):
        """Run an appending call; grow the output and repeat on capacity overflow."""
        for _ in range(8):
            rc = fn()
            B.check(rc, what)
            st = self.status.cpu()
            if int(st[1]) & B.FLAG_CAPACITY:
                out_species.ensure(int(st[0]))
                continue
            return int(st[2])
        raise B.AxpicError(f"{what}: capacity growth did not converge")

    def emit_primakoff(self, lam_in=None):
        s = self.sh
        self._ensure_ws(self.ph.n)

        def call():
            return self.lib.axpic_sample_emit(
                B.ref(self.grid), B.ref(self.cells), B.ref(self.params), B.ref(self.ph_struct),
                B.PRIMAKOFF, B.ptr(lam_in), self.step_index, self.next_id,
                B.ref(self.ax.struct()), None, B.ptr(self.hist), B.ptr(self.stats),
                B.ptr(self.status), B.ptr(self.ws), self.ws_bytes, None, s)
        self.ph_struct = self.ph.struct()
        k = self._append_call(call, self.ax, "sample_emit(primakoff)")
        self.ax.n += k
        self.next_id += k
        return k

    def emit_thermal(self, lam_in=None):
        s = self.sh
        self._ensure_ws(self.el.n)

        def call():
            return self.lib.axpic_sample_emit(
                B.ref(self.grid), B.ref(self.cells), B.ref(self.params), B.ref(self.el_struct),
                B.COMPTON | B.BREMS, B.ptr(lam_in), self.step_index, self.next_id,
                B.ref(self.ax.struct()), B.ptr(self.fb), B.ptr(self.hist), B.ptr(self.stats),
                B.ptr(self.status), B.ptr(self.ws), self.ws_bytes, None, s)
        self.el_struct = self.el.struct()
        k = self._append_call(call, self.ax, "sample_emit(thermal)")
        self.ax.n += k
        self.next_id += k
        return k

    def emit_thermal_cells(self):
        s = self.sh
        self._ensure_ws(4 * self.ncell)

        def call():
            return self.lib.axpic_sample_emit_cells(
                B.ref(self.grid), B.ref(self.cells), B.ref(self.params), B.ref(self.el_struct),
                B.ptr(self.el.off), B.ptr(self.cellw), B.COMPTON | B.BREMS, self.step_index,
                self.next_id, B.ref(self.ax.struct()), B.ptr(self.fb), B.ptr(self.hist),
                B.ptr(self.stats), B.ptr(self.status), B.ptr(self.ws), self.ws_bytes, None, s)
        self.el_struct = self.el.struct()
        k = self._append_call(call, self.ax, "sample_emit_cells")
        self.ax.n += k
        self.next_id += k
        return k

    def absorb(self, n_old: int, pabs_in=None, lam_in=None):
        s = self.sh
        self._ensure_ws(n_old)
        ax_n = self.ax.n
        self.ax.n = n_old
        try:
            def call():
                return self.lib.axpic_absorb(
                    B.ref(self.grid), B.ref(self.cells), B.ref(self.params), B.ref(self.ax_struct),
                    B.ptr(pabs_in), B.ptr(lam_in), self.step_index, self.next_id,
                    B.ref(self.ph.struct()), B.ptr(self.fb), B.ptr(self.stats), B.ptr(self.status),
                    B.ptr(self.ws), self.ws_bytes, None, s)
            self.ax_struct = self.ax.struct()
            k = self._append_call(call, self.ph, "absorb")
        finally:
            self.ax.n = ax_n
        self.ph.n += k
        self.next_id += k
        return k

    def feedback(self, moments=None, chain=None):
        self._ensure_ws(2 * self.ncell)
        B.check(self.lib.axpic_feedback(B.ref(self.grid), B.ref(self.cells), B.ref(self.params),
                                        B.ref(self.el.struct()), B.ptr(self.el.off),
                                        B.ptr(self.fb), B.ptr(moments), B.ptr(self.stats),
                                        B.ptr(self.ws), self.ws_bytes, B.ptr(chain), self.sh),
                "feedback")

    def bin_axions(self, push: bool = True):
        """Push and re-bin the axions; a push takes them out of their cell order."""
        if self.ax.n:
            B.check(self.lib.axpic_bin_cells(B.ref(self.grid), B.ref(self.ax.struct()),
                                             1 if push else 0, float(self.pdict["m_a_keV"]),
                                             self.sh), "bin_cells")
            if push:
                self.ax.off, self.ax.n_sorted = None, 0

    def sort_axions(self, chained: bool = False):
        """The axions in the canonical order (axpic_sort_cells) in the spare buffer, which
        becomes the axion buffer; its cell offsets stay in ax_off.  Chained (inside a step)
        the number kept goes to the device chain and is read back with it at the step's
        end: until then ax.n is the count before the sort (an upper bound)."""
        if not self.ax.n:
            return
        ax = self.ax
        spare = self._spare.get(B.AXION)
        if spare is None or spare.capacity < ax.n:
            spare = DeviceSpecies(B.AXION, self.dtype, self.ndim, ax.capacity, ax.w_ref,
                                  self.device)
            self._allocs += 1
        # sized for the buffer's capacity: it grows only with the buffer
        need = int(self.lib.axpic_sort_ws_bytes(B.ref(self.grid), ax.n))
        if self.sort_ws is None or self.sort_ws.numel() < need:
            need = int(self.lib.axpic_sort_ws_bytes(B.ref(self.grid), max(ax.n, ax.capacity)))
            self.sort_ws = torch.empty(need + 4096, dtype=torch.uint8, device=self.device)
            self._allocs += 1
        spare.n, spare.off, spare.n_sorted, spare.id0, spare.n_implicit = 0, None, 0, 0, 0
        spare._S = None
        B.check(self.lib.axpic_sort_cells(B.ref(self.grid), B.ref(ax.struct()), B.SORT_AUTO,
                                          B.ref(spare.struct()), B.ptr(self.ax_off),
                                          B.ptr(self.sort_status), B.ptr(self.sort_ws),
                                          self.sort_ws.numel(),
                                          B.ptr(self.chain) if chained else None, self.sh),
                "sort_cells")
        n = ax.n if chained else int(self.sort_status.cpu()[2])
        spare.n, spare.off, spare.n_sorted = n, self.ax_off, n
        self._spare[B.AXION] = ax
        self.ax = spare

    def rates(self, sp: DeviceSpecies, channel: int):
        out = torch.zeros(max(sp.n, 1), dtype=_tdtype(sp.dtype), device=self.device)
        B.check(self.lib.axpic_rates(B.ref(self.grid), B.ref(self.cells), B.ref(self.params),
                                     B.ref(sp.struct()), channel, B.ptr(out), self.sh), "rates")
        return out[: sp.n]

    def _compacted(self, sp: DeviceSpecies) -> DeviceSpecies:
        """A copy of `sp` without its particles of zero weight, in the same order, in the
        spare buffer of its kind (allocated once and reused: the replaced buffer becomes the
        next spare)."""
        spare = self._spare.get(sp.kind)
        if spare is None or spare.capacity < sp.n or spare.w_ref != sp.w_ref:
            spare = DeviceSpecies(sp.kind, self.dtype, self.ndim, sp.capacity, sp.w_ref,
                                  self.device, sp.Z, sp.A, with_p=sp.with_p,
                                  cache_p2=sp.with_p2)
            self._allocs += 1
        out = spare
        out.n, out.off, out.n_sorted, out.id0, out.n_implicit = 0, None, 0, 0, 0
        out._S = None
        self._ensure_ws(sp.n)
        B.check(self.lib.axpic_compact(B.ref(sp.struct()), B.ref(out.struct()),
                                       B.ptr(self.status), B.ptr(self.ws), self.ws_bytes, self.sh),
                "compact")
        out.n = int(self.status.cpu()[2])
        self._spare[sp.kind] = sp
        return out

    def compact_axions(self):
        if self.ax.n:
            self.ax = self._compacted(self.ax)

    def compact_photons(self):
        """Photons converted whole by the Primakoff operator keep a zero weight; under
        a->gamma new photons keep arriving and are converted back, so the dead ones pile
        up.  The per-cell offsets of the input photons are not used by any operator."""
        if self.ph.n:
            self.ph = self._compacted(self.ph)

    def diag(self):
        self._ensure_ws(self.ax.n)
        B.check(self.lib.axpic_diag(B.ref(self.ax.struct()), float(self.pdict["m_a_keV"]),
                                    B.ptr(self.diag_out), B.ptr(self.ws),
                                    self.ws_bytes, self.sh), "diag")
        v = self.diag_out.cpu().tolist()
        return dict(N_a=v[0], U_a=v[1])

    def equilibrium(self, t_steps: float = 0.0, sp: Optional[DeviceSpecies] = None) -> Dict:
        """The library's FP64 equilibrium check (axpic_equilibrium) of the axions (or of
        `sp`) at the current temperature field (the cell state is recomputed first): per
        histogram bin the population's number, energy and sum of squared weights, the
        equilibrium number and energy, the recursion content after t_steps steps (<= 0:
        its fixed point) and the residual z; arrays of nbins + 2 (underflow, overflow
        last)."""
        sp = self.ax if sp is None else sp
        self.cell_state()
        nbh = self.pdict["hist_nbins"] + 2
        out = torch.zeros(7 * nbh, dtype=torch.float64, device=self.device)
        need = int(self.lib.axpic_equilibrium_ws_bytes(sp.n, self.ncell,
                                                       self.pdict["hist_nbins"]))
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        B.check(self.lib.axpic_equilibrium(B.ref(self.grid), B.ref(self.cells),
                                           B.ref(self.params), B.ref(sp.struct()),
                                           float(t_steps), B.ptr(out), B.ptr(ws), ws.numel(),
                                           self.sh), "equilibrium")
        v = out.cpu().numpy()
        return {k: v[i * nbh:(i + 1) * nbh].copy() for i, k in enumerate(B.EQ_FIELDS)}

    # -------------------------------------------------------------- one step
    def step(self):
        """One time step.  The sort and the appending calls are chained on the device
        (counts and the next id stay there), so the step reads back the chain's words once
        at its end; after an overflow the buffer named by the failing call is grown and the
        calls are repeated from it on (the skipped ones modified nothing)."""
        p = self.pdict
        self.bin_axions(push=True)
        if self.sort and not self.sort_chained:
            self.sort_axions(chained=False)          # the kept count is now ax.n
        # the chain's words before the first chained call (a chained sort rewrites the
        # axion count and the start-of-step word on the device)
        self._chain_np[:] = (self.ax.n, self.ph.n, self.next_id, 0, self.ax.n)
        self.chain.copy_(self.chain_host, non_blocking=True)
        if self.sort and self.sort_chained:
            self.sort_axions(chained=True)
        if p["T_mode"] == 2:
            self.cell_state()
        if self.need_feedback:
            self.fb.zero_()
        n_ax0 = self.ax.n
        if self.grow_ahead:
            self.ax.ensure(self.ax.n + 2 * self._last_new[0] + 4096)
            if p["inverse"] and p["channels"] & B.PRIMAKOFF:
                self.ph.ensure(self.ph.n + 2 * self._last_new[1] + 1024)
        self._ensure_ws(max(self.el.capacity, self.ph.capacity, self.ax.capacity, 4 * self.ncell))
        S = self.surrogate
        lam = pab = lag = None
        if S and self.surrogate_mode == "table":
            # one network pass per cell and node; the particles interpolate
            need = p["channels"] & B.PRIMAKOFF
            if p["inverse"] and n_ax0 > 0:
                need |= p["channels"] & (B.COMPTON | B.BREMS)
            if need:
                self._tab = S.table(self, need, out=self._tab)

            def srates(sp, ch):
                return S.rates_table(self, sp, ch, self._tab, fallback=self.fallback)
        else:
            def srates(sp, ch):
                return S.rates(self, sp, ch, fallback=self.fallback)
        if S and p["channels"] & B.PRIMAKOFF:
            lam = srates(self.ph, B.PRIMAKOFF)
        if S and p["inverse"] and n_ax0 > 0:
            n_now = self.ax.n
            self.ax.n = n_ax0
            try:
                if p["channels"] & (B.COMPTON | B.BREMS):
                    pab = srates(self.ax, B.COMPTON | B.BREMS)
                if p["channels"] & B.PRIMAKOFF:
                    lag = srates(self.ax, B.PRIMAKOFF)
            finally:
                self.ax.n = n_now
        n_ph0, id0 = self.ph.n, self.next_id
        st = self.status_ops
        sh, g, c, prm, ch = self.sh, B.ref(self.grid), B.ref(self.cells), B.ref(self.params), \
            B.ptr(self.chain)

        def op_prim():
            return self.lib.axpic_sample_emit(
                g, c, prm, B.ref(self.ph.struct()), B.PRIMAKOFF, B.ptr(lam), self.step_index, id0,
                B.ref(self.ax.struct()), None, B.ptr(self.hist), B.ptr(self.stats), B.ptr(st[0]),
                B.ptr(self.ws), self.ws_bytes, ch, sh)

        def op_therm():
            if self.thermal == "cells":
                return self.lib.axpic_sample_emit_cells(
                    g, c, prm, B.ref(self.el.struct()), B.ptr(self.el.off), B.ptr(self.cellw),
                    B.COMPTON | B.BREMS, self.step_index, id0, B.ref(self.ax.struct()),
                    B.ptr(self.fb), B.ptr(self.hist), B.ptr(self.stats), B.ptr(st[1]),
                    B.ptr(self.ws), self.ws_bytes, ch, sh)
            return self.lib.axpic_sample_emit(
                g, c, prm, B.ref(self.el.struct()), B.COMPTON | B.BREMS, None, self.step_index,
                id0, B.ref(self.ax.struct()), B.ptr(self.fb), B.ptr(self.hist), B.ptr(self.stats),
                B.ptr(st[1]), B.ptr(self.ws), self.ws_bytes, ch, sh)

        def op_abs():
            axs = self.ax.struct()
            axs.n = n_ax0
            return self.lib.axpic_absorb(
                g, c, prm, B.ref(axs), B.ptr(pab), B.ptr(lag), self.step_index, id0,
                B.ref(self.ph.struct()), B.ptr(self.fb), B.ptr(self.stats), B.ptr(st[2]),
                B.ptr(self.ws), self.ws_bytes, ch, sh)

        def op_fb():
            return self.lib.axpic_feedback(g, c, prm, B.ref(self.el.struct()), B.ptr(self.el.off),
                                           B.ptr(self.fb), None, B.ptr(self.stats),
                                           B.ptr(self.ws), self.ws_bytes, ch, sh)
        ops = []
        if p["channels"] & B.PRIMAKOFF:
            ops.append((op_prim, 0, self.ax))
        if p["channels"] & (B.COMPTON | B.BREMS):
            ops.append((op_therm, 1, self.ax))
        if p["inverse"] and n_ax0 > 0:
            ops.append((op_abs, 2, self.ph))
        if self.need_feedback:
            ops.append((op_fb, -1, None))
        first = 0
        for _ in range(8):
            for fn, _, _ in ops[first:]:
                B.check(fn(), "step")
            cw = self.chain.cpu()
            if int(cw[3]) == 0:
                break
            sts = st.cpu()
            # what the successful calls appended is on the device: the growth must keep it
            self.ax.n, self.ph.n = int(cw[0]), int(cw[1])
            for k, (fn, slot, sp) in enumerate(ops):
                if slot >= 0 and int(sts[slot][1]) & B.FLAG_CAPACITY:
                    sp.ensure(int(sts[slot][0]))
                    first = k
                    break
            else:
                raise B.AxpicError("chained step: skip flag without a capacity overflow")
            self.chain[3].zero_()
        else:
            raise B.AxpicError("chained step: capacity growth did not converge")
        self.ax.n, self.ph.n, self.next_id = int(cw[0]), int(cw[1]), int(cw[2])
        n_ax0 = int(cw[B.CHAIN_AX_START])
        if self.ax.off is not None:              # the sorted prefix: what the sort kept
            self.ax.n_sorted = n_ax0
        self._last_new = (self.ax.n - n_ax0, self.ph.n - n_ph0)
        self.step_index += 1
        if self.compact_every and self.step_index % self.compact_every == 0:
            if not self.sort:            # sorting drops the axions of zero weight every step
                self.compact_axions()
            if p["inverse"] and p["channels"] & B.PRIMAKOFF:
                self.compact_photons()

    def hist_np(self):
        nb = self.pdict["hist_nbins"] + 2
        return self.hist.cpu().numpy().reshape(3, nb)

    def stats_dict(self):
        v = self.stats.cpu().numpy()
        return {n: float(v[i]) for i, n in enumerate(B.ST_NAMES)}
