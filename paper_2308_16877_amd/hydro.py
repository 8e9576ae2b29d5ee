"""Lagrangian Sedov blast on the library's hydro kernels, with TAF and
perforation on its hourglass and EOS regions across timesteps.

`Hydro` owns the device state (torch tensors in the C layout of
include/hpac.h) and calls hpac_hydro_init / hpac_hydro_step; every step runs
in the HIP kernels.
"""
import ctypes

import numpy as np
import torch

from . import hpac

# Workload constants of the blast: unit cube, ideal gas gamma = 1.4, unit
# density, full-space energy 1 (one eighth in the octant's origin element).
DEFAULTS = dict(side=1.0, gamma=1.4, cq=1.5, cl=0.25, khg=0.1, cfl=0.3, growth=1.1, dvmax=0.1, dt0=1e-7)


def sedov_origin_energy(n, side=1.0, energy=1.0):
    """Specific energy of the origin element that holds an eighth of
    `energy` (the octant of a full-space blast) at unit density."""
    return (energy / 8.0) / (side / n) ** 3


class Tech:
    """Technique of the hydro regions: eos / hg = (history, prediction,
    threshold[, level]) for TAF, level "wave" (default), "thread" or "block";
    perfo = (kind, param, items_per_lane) for the hourglass region."""

    def __init__(self, eos=None, hg=None, perfo=None):
        self.eos, self.hg, self.perfo = eos, hg, perfo
        t = hpac.hpac_hydro_tech(eos_level=hpac.LEVEL_WAVE, hg_level=hpac.LEVEL_WAVE)
        if eos:
            t.eos_history, t.eos_prediction, t.eos_threshold = int(eos[0]), int(eos[1]), float(eos[2])
            t.eos_level = hpac._level(eos[3]) if len(eos) > 3 else hpac.LEVEL_WAVE
        if hg:
            t.hg_history, t.hg_prediction, t.hg_threshold = int(hg[0]), int(hg[1]), float(hg[2])
            t.hg_level = hpac._level(hg[3]) if len(hg) > 3 else hpac.LEVEL_WAVE
        if perfo:
            kind = hpac.PERFO_KINDS[perfo[0]] if isinstance(perfo[0], str) else int(perfo[0])
            t.perfo_kind, t.perfo_param, t.perfo_items_per_lane = kind, int(perfo[1]), int(perfo[2])
        self.c = t


class Hydro:
    FIELDS = ("mnode", "e", "p", "q", "c", "vol", "mass", "force")

    def __init__(self, n, e_origin=None, tech=None, device="cuda:0", **par):
        self.n = int(n)
        self.par = dict(DEFAULTS, **par)
        self.tech = tech or Tech()
        E, Nn = self.n ** 3, (self.n + 1) ** 3
        self.E, self.Nn = E, Nn
        self.W = hpac.hpac_hydro_waves(self.n)
        f32 = dict(dtype=torch.float32, device=device)
        self.x = torch.zeros(3, Nn, **f32)
        self.u = torch.zeros(3, Nn, **f32)
        self.unew = torch.zeros(3, Nn, **f32)
        self.mnode = torch.zeros(Nn, **f32)
        for f in ("e", "p", "q", "c", "vol", "mass"):
            setattr(self, f, torch.zeros(E, **f32))
        self.force = torch.zeros(24, E, **f32)
        t = self.tech
        i32 = dict(dtype=torch.int32, device=device)
        # decision-group state: one entry per element covers every level
        self.weos = torch.zeros(max(t.eos[0], 1) * 4, E, **f32) if t.eos else None
        self.rho_eos = torch.zeros(E, **i32) if t.eos else None
        self.z_eos = torch.zeros(E, **i32) if t.eos else None
        self.whg = torch.zeros(max(t.hg[0], 1) * 24, E, **f32) if t.hg else None
        self.rho_hg = torch.zeros(E, **i32) if t.hg else None
        self.z_hg = torch.zeros(E, **i32) if t.hg else None
        self.clock = torch.zeros(2, dtype=torch.float64, device=device)
        self.dt_partials = torch.zeros(hpac.hpac_hydro_partials(self.n), dtype=torch.float64, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.dec_eos = torch.zeros(E, dtype=torch.int8, device=device)
        self.dec_hg = torch.zeros(E, dtype=torch.int8, device=device)
        self.params = hpac.hpac_hydro_params(n=self.n, **self.par)
        self.steps = 0
        self._bind()
        e0 = sedov_origin_energy(self.n, self.par["side"]) if e_origin is None else e_origin
        hpac.hpac_hydro_init(self.params, e0, self.state)

    def _bind(self):
        s = hpac.hpac_hydro_state()
        for d in range(3):
            s.x[d] = self.x[d].data_ptr()
            s.u[d] = self.u[d].data_ptr()
            s.unew[d] = self.unew[d].data_ptr()
        for f in self.FIELDS + ("weos", "rho_eos", "z_eos", "whg", "rho_hg", "z_hg", "clock", "dt_partials",
                                "status"):
            t = getattr(self, f)
            setattr(s, f, t.data_ptr() if t is not None else None)
        self.state = s

    def step(self, record=False, stream=None, noalloc=False):
        """One timestep (index = number of steps taken so far); noalloc: by
        hpac_hydro_step_noalloc, the time-step partials in the library's own
        scratch array."""
        fn = hpac.hpac_hydro_step_noalloc if noalloc else hpac.hpac_hydro_step
        fn(self.params, self.tech.c, self.steps, self.state,
           self.dec_eos if record else None, self.dec_hg if record else None, stream)
        self._swap_velocities()
        self.steps += 1

    def _swap_velocities(self):
        self.u, self.unew = self.unew, self.u
        for d in range(3):  # element-wise: ctypes array fields are views of the struct
            self.state.u[d] = self.u[d].data_ptr()
            self.state.unew[d] = self.unew[d].data_ptr()

    def run(self, steps, stream=None):
        """`steps` timesteps issued by the library's own loop (no records)."""
        hpac.hpac_hydro_run(self.params, self.tech.c, self.steps, steps, self.state, stream)
        if steps % 2:
            self._swap_velocities()
        self.steps += steps

    def check(self, stream=None):
        """Raises hpac.HpacError (HPAC_ENUMERIC) if a step so far left the
        numeric domain (a non-positive element volume or time step)."""
        hpac.hpac_hydro_check(self.state, stream)

    def time(self):
        return float(self.clock[0])

    def origin_energy(self):
        """The quantity of interest: specific energy of the origin element."""
        return float(self.e[0])

    def energy(self):
        """(internal, kinetic) energy, summed in FP64."""
        ie = float((self.mass.double() * self.e.double()).sum())
        ke = float((0.5 * self.mnode.double() * (self.u.double() ** 2).sum(0)).sum())
        return ie, ke

    def numpy_state(self):
        """Host copy of the state (float64 arrays) in the oracle's layout."""
        out = {}
        for f in ("x", "u", "mnode", "e", "p", "q", "c", "vol", "mass", "force", "weos", "whg"):
            t = getattr(self, f)
            out[f] = t.double().cpu().numpy() if t is not None else None
        for f in ("rho_eos", "z_eos", "rho_hg", "z_hg"):
            t = getattr(self, f)
            out[f] = t.cpu().numpy() if t is not None else None
        out["clock"] = self.clock.cpu().numpy()
        return out
