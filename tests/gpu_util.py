"""Helpers for the GPU parity tests: build matching oracle and device runs from
the same synthetic configuration."""
import numpy as np

import paper_2307_11107_amd as apic
from oracle.pic import Config, Simulation, Species


def species_pair(w, electrons=True, ions=True, weight=0.0, n_macro=None):
    """Species definitions (device, oracle) for a workload dict."""
    n = w["n_macro"] if n_macro is None else n_macro
    dev, ora = [], []
    if electrons:
        dev.append(apic.species(-1.0, 1.0, 1.0, 1.0, 0.0, weight, n))
        ora.append(Species(q=-1.0, m=1.0, T=1.0, n=1.0, n_macro=n, weight=weight))
    if ions:
        dev.append(apic.species(1.0, w["mi"], w["Ti"], 1.0, 0.0, weight, n))
        ora.append(Species(q=1.0, m=w["mi"], T=w["Ti"], n=1.0, n_macro=n, weight=weight))
    return dev, ora


def make_pair(w, precision, inject=True, frozen=False, electrons=True, ions=True, weight=0.0,
              n_macro=None, n_bins=0, sort_every=0, poisson_tol=0.0, capacity=0, boltzmann=False,
              conservative=False):
    dev_sp, ora_sp = species_pair(w, electrons, ions, weight, n_macro)
    if capacity:
        for s in dev_sp:
            s.capacity = capacity
    cfg = apic.grain_cfg(w["alpha"], w["n1"], w["n2"], dev_sp, x1_out=w["x1_out"], wce=w["wce"],
                         kappa=w["kappa"], phi_grain=-2.5, phi_out=0.0, dt=w["dt"], n_bins=n_bins,
                         seed=w["seed"])
    ctx = apic.apic_init([cfg], apic.opts(precision=precision, inject=inject, frozen_field=frozen,
                                          sort_every=sort_every, poisson_tol=poisson_tol,
                                          boltzmann_electrons=boltzmann, conservative_poisson=conservative))
    ocfg = Config(alpha=w["alpha"], n1=w["n1"], n2=w["n2"], x1_out=w["x1_out"], wce=w["wce"],
                  kappa=w["kappa"], dt=w["dt"], n_bins=n_bins, seed=w["seed"], species=ora_sp,
                  boltzmann=boltzmann, conservative=conservative)
    sim = Simulation(ocfg)
    sim.inject_enabled = inject
    sim.frozen = frozen
    return ctx, sim


def shape_of(w):
    return (w["n2"] + 1, w["n1"] + 1)


def particle_error(dev, ora, grid, vscale):
    """Per-particle relative error |d| / (|ref| + scale): positions with the local
    cell size as scale, velocities with the thermal speed.  Returns the array of
    per-particle maxima (over the five components); particles are matched by id."""
    common, ia, ib = np.intersect1d(dev["id"], ora["id"], return_indices=True)
    out = np.zeros(len(common))
    for k, scale in (("x1", grid.h1), ("x2", grid.h2), ("vR", vscale), ("vZ", vscale), ("vT", vscale)):
        a, b = dev[k][ia], ora[k][ib]
        out = np.maximum(out, np.abs(a - b) / (np.abs(b) + scale))
    return out, len(common)
