"""Python binding of libapic.so, the MI355X (gfx950) particle loop of the
aspherical particle-in-cell method (arXiv 2307.11107).

Argument marshalling only: every step of the loop runs in the HIP kernels behind
the C ABI of include/apic.h.  The functions carry the ABI's names; arrays are
numpy arrays on the host.  A missing library raises instead of falling back to
anything else.
"""
import ctypes as C

import numpy as np

from . import _abi
from ._abi import (APIC_FP32_SPLIT, APIC_FP64, APIC_OK, APIC_EINVAL, APIC_ERANGE, APIC_ENOMEM,
                   APIC_EDEVICE, APIC_ESTATE, apic_species, apic_grain_cfg, apic_opts)

_lib = None


class ApicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_abi.ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    """The loaded libapic.so (loaded on first use)."""
    global _lib
    if _lib is None:
        _lib = _abi.load()
    return _lib


def _check(rc, ctx=None):
    if rc != APIC_OK:
        msg = lib().apic_last_error(ctx)
        raise ApicError(rc, msg.decode() if msg else "")


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def species(q, m, T=1.0, n=1.0, e_bind=0.0, weight=0.0, n_macro=0, capacity=0):
    return apic_species(q, m, T, n, e_bind, weight, int(n_macro), int(capacity))


def grain_cfg(alpha, n1, n2, species_list, x1_out=-0.1, wce=0.0, kappa=1.0, phi_grain=-2.5,
              phi_out=0.0, dt=0.05, n_bins=0, seed=0):
    c = apic_grain_cfg()
    c.alpha, c.wce, c.kappa, c.x1_out = alpha, wce, kappa, x1_out
    c.phi_grain, c.phi_out, c.dt = phi_grain, phi_out, dt
    c.n1, c.n2, c.n_bins = int(n1), int(n2), int(n_bins)
    c.n_species = len(species_list)
    c.seed = int(seed)
    for k, s in enumerate(species_list):
        c.sp[k] = s
    return c


def opts(precision=APIC_FP32_SPLIT, inject=True, frozen_field=False, sort_every=0,
         poisson_tol=0.0, poisson_max_cycles=0, stream=None, autotune=False, boltzmann_electrons=False,
         conservative_poisson=False):
    o = apic_opts()
    o.boltzmann_electrons = int(boltzmann_electrons)
    o.conservative_poisson = int(conservative_poisson)
    o.precision, o.inject, o.frozen_field, o.sort_every = precision, int(inject), int(frozen_field), sort_every
    o.poisson_tol, o.poisson_max_cycles = poisson_tol, poisson_max_cycles
    o.autotune = int(autotune)
    o.stream = stream
    return o


# ---------------------------------------------------------------- ABI calls
def apic_init(cfgs, options=None):
    """Creates a context for a list of grain configurations; returns its handle."""
    arr = (apic_grain_cfg * len(cfgs))(*cfgs)
    h = C.c_void_p()
    rc = lib().apic_init(arr, len(cfgs), C.byref(options) if options is not None else None, C.byref(h))
    _check(rc, None)
    return h


def apic_inject(ctx, grain, sp, x1=None, x2=None, vR=None, vZ=None, vTheta=None):
    """Explicit particles (float64 arrays), or the volume load when x1 is None."""
    if x1 is None:
        _check(lib().apic_inject(ctx, grain, sp, -1, None, None, None, None, None), ctx)
        return
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x1, x2, vR, vZ, vTheta)]
    n = len(arrs[0])
    if any(len(a) != n for a in arrs):
        raise ValueError("particle arrays differ in length")
    _check(lib().apic_inject(ctx, grain, sp, n, *[_dptr(a) for a in arrs]), ctx)


def apic_inject_noalloc(ctx, grain, sp, x1, x2, vR, vZ, vTheta):
    """Explicit particles (float64 arrays) staged without device allocation."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x1, x2, vR, vZ, vTheta)]
    n = len(arrs[0])
    if any(len(a) != n for a in arrs):
        raise ValueError("particle arrays differ in length")
    _check(lib().apic_inject_noalloc(ctx, grain, sp, n, *[_dptr(a) for a in arrs]), ctx)


def apic_step(ctx, n_steps=1):
    _check(lib().apic_step(ctx, int(n_steps)), ctx)


def apic_solve_poisson(ctx, grain, rho=None, shape=None):
    """Solves eqs. (6)-(7); rho (nodes, [i2, i1] or flat) or None (deposit the
    particles).  Returns phi as a flat float64 array of (n1+1)(n2+1)."""
    if shape is None:
        raise ValueError("shape=(n2+1, n1+1) is required")
    out = np.zeros(shape[0] * shape[1])
    r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).ravel()
    if r is not None and r.size != out.size:
        raise ValueError("rho has the wrong size")
    _check(lib().apic_solve_poisson(ctx, grain, _dptr(r), _dptr(out)), ctx)
    return out.reshape(shape)


def apic_tallies(ctx, grain, n_species, n_bins):
    t = _abi.apic_tally()
    nb = n_species * n_bins
    bufs = {k: np.zeros(nb) for k in ("charge", "pR", "pZ", "L", "energy")}
    count = np.zeros(nb, dtype=np.uint64)
    for k, v in bufs.items():
        setattr(t, k, _dptr(v))
    t.count = count.ctypes.data_as(C.POINTER(C.c_uint64))
    _check(lib().apic_tallies(ctx, grain, C.byref(t)), ctx)
    ns = t.n_species
    out = {k: v.reshape(n_species, n_bins) for k, v in bufs.items()}
    out["count"] = count.reshape(n_species, n_bins).astype(np.int64)
    for k in ("injected", "absorbed", "escaped", "resident", "particle_steps"):
        out[k] = np.array([getattr(t, k)[s] for s in range(ns)], dtype=np.int64)
    out["weight"] = np.array([t.weight[s] for s in range(ns)])
    out["steps"] = int(t.steps)
    out["F_el_sum"] = float(t.F_el_sum)
    out["unconverged_solves"] = int(t.unconverged_solves)
    return out


def apic_particles(ctx, grain, sp, cap):
    """Live particles of one species sorted by id: dict of float64 arrays + id."""
    bufs = {k: np.zeros(max(cap, 1)) for k in ("x1", "x2", "vR", "vZ", "vT")}
    ids = np.zeros(max(cap, 1), dtype=np.int64)
    n = C.c_int64()
    rc = lib().apic_particles(ctx, grain, sp, cap, *[_dptr(bufs[k]) for k in ("x1", "x2", "vR", "vZ", "vT")],
                              ids.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(n))
    _check(rc, ctx)
    m = n.value
    out = {k: v[:m].copy() for k, v in bufs.items()}
    out["id"] = ids[:m].copy()
    return out


def apic_schedule(ctx):
    """The context's launch schedule: dict push_wg_per_cu, tile_log2, sort_every, tuned."""
    sc = _abi.apic_sched()
    _check(lib().apic_schedule(ctx, C.byref(sc)), ctx)
    return {k: int(getattr(sc, k)) for k in ("push_wg_per_cu", "tile_log2", "sort_every", "tuned")}


def apic_fields(ctx, grain, shape):
    phi = np.zeros(shape[0] * shape[1])
    rho = np.zeros(shape[0] * shape[1])
    _check(lib().apic_fields(ctx, grain, _dptr(phi), _dptr(rho)), ctx)
    return phi.reshape(shape), rho.reshape(shape)


def apic_surface_field(ctx, grain, n2):
    """Normal field E_n on the grain at the nodes i2 = 0..n2 (surface charge = eps0 E_n)."""
    en = np.zeros(n2 + 1)
    _check(lib().apic_surface_field(ctx, grain, _dptr(en)), ctx)
    return en


def apic_set_profiling(ctx, on=True):
    _check(lib().apic_set_profiling(ctx, int(on)), ctx)


def apic_timing(ctx):
    t = _abi.apic_kernel_times()
    _check(lib().apic_timing(ctx, C.byref(t)), ctx)
    return {k: getattr(t, k) for k, _ in t._fields_}


def apic_free(ctx):
    if ctx:
        lib().apic_free(ctx)


def apic_last_error(ctx=None):
    m = lib().apic_last_error(ctx)
    return m.decode() if m else ""
