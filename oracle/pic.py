"""Plain FP64 particle-in-cell time loop of the aspherical PIC method.

Oracle module: test infrastructure only.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark import it; the product path never does.

It follows the paper's Sections 1-2 in their own order: macro-particles with the
species' q/m; charge weighted to the nodes with the volume element (eq. 5);
Poisson's equation (eqs. 6-7) solved by LU with fixed potentials on the grain
and the outer boundary; the field from eq. (10); the equations of motion (9)
advanced by leapfrog; particles absorbed by the grain transfer charge, momentum,
angular momentum and kinetic plus binding energy at the impact point; particles
leaving through the outer boundary are removed; a Maxwellian flux is injected
through the outer boundary.  Diagnostics: the electric force on the grain from
the surface field, and the surface charge density from the normal field.

With Config.conservative the field solve uses the conservative (finite-element)
form of poisson.assemble_fe, its right-hand side the node charges.
With Config.boltzmann the electrons are not moved: their density is n0 exp(phi)
(Section 2, last paragraph; the physical sign) and the field solve is the
nonlinear one of poisson.solve_boltzmann, started from the current potential.

Readings where the paper is silent (all shared with the device implementation,
which is written separately):
  * units: R0, 1/omega_pe, v_te, Te/e, n0, me, e; kappa = lambda_De / R0;
    Lap(phi) = -(1/kappa^2) sum_s q_s n_s;
  * a species' macro-particle weight is w_s = n_s V / N_s (V the domain volume,
    N_s the initial load), unless a weight is given explicitly;
  * initial load: positions uniform in physical volume (x2 by rejection on the
    marginal r_out^3 - r_in^3, then r^3 uniform), velocities Maxwellian with
    thermal speed sqrt(T_s/m_s), taken as v^{-1/2};
  * injection: per step N = Gamma_s A_out kappa dt / w_s with the one-way flux
    Gamma_s = n_s sqrt(T_s / (2 pi m_s)), carried in a 2^-32 fixed-point
    accumulator so the counts are exact integers; x2 drawn with density
    proportional to eq. (4) at x1_out; velocity: inward normal component
    Rayleigh(sqrt(T_s/m_s)), two tangential components normal(0, T_s/m_s); the
    particle is then moved straight on for a fraction U (uniform) of a step;
  * random numbers: Philox4x32-10, key (lo32(seed), hi32(seed) + grain),
    counter (stream, species | purpose << 8, slot, draw); stream = step index
    for injection, 0xFFFFFFFF for the initial load; purposes 1/2 = load
    position/velocity, 3/4 = injection position/velocity;
  * tallies: per species and per x2-bin of the impact point: count, charge,
    R- and Z-momentum, angular momentum about the axis, kinetic + binding
    energy, each multiplied by the macro-particle weight;
  * electric force on the grain: Maxwell stress of a conductor,
    F_Z = integral of E_n^2 / 2 * n_Z dA over x1 = -1, trapezoid over the nodes.
"""
from dataclasses import dataclass, field as dc_field

import numpy as np

from . import geometry as geo
from . import grid as gridmod
from . import poisson
from . import field
from . import mover
from .philox import philox4x32_10, to_unit, key_for

LOAD_STREAM = 0xFFFFFFFF
P_LOAD_POS, P_LOAD_VEL, P_INJ_POS, P_INJ_VEL = 1, 2, 3, 4
MAX_ATTEMPTS = 64
TWO32 = 1 << 32


@dataclass
class Species:
    q: float                 # charge, units of e
    m: float                 # mass, units of me
    T: float = 1.0           # temperature, units of Te
    n: float = 1.0           # unperturbed density, units of n0
    e_bind: float = 0.0      # energy deposited per absorbed particle besides kinetic
    n_macro: int = 0         # initial volume load
    weight: float = 0.0      # macro-particle weight (0: n V / n_macro)


@dataclass
class Config:
    alpha: float
    n1: int
    n2: int
    x1_out: float = -0.1
    wce: float = 0.0              # omega_ce / omega_pe
    kappa: float = 1.0            # lambda_De / R0
    phi_grain: float = -2.5
    phi_out: float = 0.0
    dt: float = 0.05
    n_bins: int = 0               # 0: n2
    seed: int = 0
    grain: int = 0
    species: list = dc_field(default_factory=list)
    boltzmann: bool = False       # electrons as n0 exp(phi), not moved (species: the moved ones)
    conservative: bool = False    # field solve on the conservative (finite-element) form


def _max_sampled(f, npts=4097):
    x2 = np.linspace(-1.0, 1.0, npts)
    return 1.0001 * float(np.max(f(x2)))


class Simulation:
    def __init__(self, cfg, vacuum_field=True):
        """vacuum_field=False leaves the potential unset (the caller sets it with
        set_phi) and factorises the Poisson operator only when a solve is first
        asked for: a large grid's factorisation takes minutes."""
        if not geo.check_alpha(cfg.alpha, cfg.x1_out):
            raise ValueError("need |alpha| < 1/4 and -1 < x1_out < 0")
        self.cfg = cfg
        self.grid = gridmod.Grid(cfg.n1, cfg.n2, cfg.x1_out, cfg.alpha)
        self.n_bins = cfg.n_bins if cfg.n_bins > 0 else cfg.n2
        self.vol = gridmod.node_volumes(self.grid)
        self.V = float(np.sum(self.vol))
        self.A_out = gridmod.outer_area(self.grid)
        self._solver = None
        self._A = None
        self.key = key_for(cfg.seed, cfg.grain)
        a = cfg.alpha
        self.M_vol = _max_sampled(lambda x2: geo.r_of(cfg.x1_out, x2, a) ** 3 - geo.r_of(-1.0, x2, a) ** 3)
        self.M_area = _max_sampled(lambda x2: geo.dA_dx2(cfg.x1_out, x2, a))
        ns = len(cfg.species)
        self.w = []
        self.inj_inc = []
        for sp in cfg.species:
            w = sp.weight if sp.weight > 0 else (sp.n * self.V / sp.n_macro if sp.n_macro > 0 else 0.0)
            self.w.append(w)
            flux = sp.n * np.sqrt(sp.T / (2.0 * np.pi * sp.m))
            n_real = flux * self.A_out * cfg.kappa * cfg.dt / w if w > 0 else 0.0
            self.inj_inc.append(int(round(n_real * TWO32)))
        self.inj_acc = [0] * ns
        self.parts = [self._empty() for _ in range(ns)]
        self.next_id = [0] * ns
        self.step_index = 0
        self.inject_enabled = True
        self.frozen = False
        nb = self.n_bins
        self.tally = {k: np.zeros((ns, nb)) for k in ("charge", "pR", "pZ", "L", "energy")}
        self.tally["count"] = np.zeros((ns, nb), dtype=np.int64)
        self.injected = np.zeros(ns, dtype=np.int64)
        self.absorbed = np.zeros(ns, dtype=np.int64)
        self.escaped = np.zeros(ns, dtype=np.int64)
        self.F_el_sum = 0.0
        self.diag_steps = 0
        self.phi = self.phi1 = self.phi2 = None
        if vacuum_field:
            if cfg.conservative:
                self._A = poisson.assemble_fe(self.grid)
                self.set_phi(poisson.solve_fe(self.grid, self._A, np.zeros(self.grid.shape), cfg.kappa,
                                              cfg.phi_grain, cfg.phi_out))
            else:
                self.set_phi(self.solver.solve(np.zeros(self.grid.shape), cfg.phi_grain, cfg.phi_out))

    @property
    def solver(self):
        if self._solver is None:
            self._solver = poisson.PoissonSolver(self.grid)
        return self._solver

    # ------------------------------------------------------------------ state
    @staticmethod
    def _empty():
        z = np.zeros(0)
        return {"x1": z, "x2": z, "vR": z, "vZ": z, "vT": z, "id": np.zeros(0, dtype=np.int64)}

    def set_particles(self, s, x1, x2, vR, vZ, vT, ids=None):
        """Explicit particles (ids 0..n-1 unless given), replacing species s."""
        n = len(x1)
        idv = np.arange(n, dtype=np.int64) if ids is None else np.array(ids, dtype=np.int64)
        self.parts[s] = {"x1": np.array(x1, dtype=np.float64), "x2": np.array(x2, dtype=np.float64),
                         "vR": np.array(vR, dtype=np.float64), "vZ": np.array(vZ, dtype=np.float64),
                         "vT": np.array(vT, dtype=np.float64), "id": idv}
        self.next_id[s] = int(idv.max()) + 1 if n else 0

    def particles(self, s):
        """Copy of species s sorted by particle id."""
        p = self.parts[s]
        o = np.argsort(p["id"], kind="stable")
        return {k: v[o] for k, v in p.items()}

    def resident(self, s):
        return len(self.parts[s]["x1"])

    # ------------------------------------------------------------------ load
    def load(self, s, n=None, slots=None):
        """Initial volume load of species s (n defaults to n_macro).  With
        `slots`, only the particles of those load indices are drawn (each
        particle's draws depend on its own index alone), with ids = slots."""
        sp = self.cfg.species[s]
        n = sp.n_macro if n is None else n
        a, xo = self.cfg.alpha, self.cfg.x1_out
        slot = np.arange(n, dtype=np.uint64) if slots is None else np.asarray(slots, dtype=np.uint64)
        n = len(slot)
        x2 = np.zeros(n)
        r3 = np.zeros(n)
        todo = np.ones(n, dtype=bool)
        for k in range(MAX_ATTEMPTS):
            u0, u1, u2, _ = philox4x32_10(LOAD_STREAM, s | (P_LOAD_POS << 8), slot, k, *self.key)
            cx2 = -1.0 + 2.0 * to_unit(u0)
            rin3 = geo.r_of(-1.0, cx2, a) ** 3
            rout3 = geo.r_of(xo, cx2, a) ** 3
            acc = to_unit(u1) * self.M_vol <= (rout3 - rin3)
            take = todo & (acc | (k == MAX_ATTEMPTS - 1))
            x2[take] = cx2[take]
            r3[take] = (rin3 + to_unit(u2) * (rout3 - rin3))[take]
            todo &= ~take
            if not todo.any():
                break
        r = np.cbrt(r3)
        x1 = geo.x1_of(r, x2, a)
        u0, u1, u2, u3 = philox4x32_10(LOAD_STREAM, s | (P_LOAD_VEL << 8), slot, 0, *self.key)
        sig = np.sqrt(sp.T / sp.m)
        g0 = np.sqrt(-2.0 * np.log(to_unit(u0)))
        g1 = np.sqrt(-2.0 * np.log(to_unit(u2)))
        vR = sig * g0 * np.cos(2.0 * np.pi * to_unit(u1))
        vZ = sig * g0 * np.sin(2.0 * np.pi * to_unit(u1))
        vT = sig * g1 * np.cos(2.0 * np.pi * to_unit(u3))
        self.set_particles(s, x1, x2, vR, vZ, vT, ids=None if slots is None else slot.astype(np.int64))

    # ------------------------------------------------------------------ field
    def deposit(self, x1, x2):
        """Bilinear (cloud-in-cell) weights of the positions summed at the nodes."""
        g = self.grid
        i1, i2, f1, f2 = field.locate(x1, x2, g)
        dep = np.zeros(g.shape)
        np.add.at(dep, (i2, i1), (1 - f1) * (1 - f2))
        np.add.at(dep, (i2, i1 + 1), f1 * (1 - f2))
        np.add.at(dep, (i2 + 1, i1), (1 - f1) * f2)
        np.add.at(dep, (i2 + 1, i1 + 1), f1 * f2)
        return dep

    def densities(self, deps):
        return [self.w[s] * deps[s] / self.vol for s in range(len(deps))]

    def solve_field(self, deps):
        if self.cfg.conservative:
            # the node charges themselves are the right-hand side
            if self._A is None:
                self._A = poisson.assemble_fe(self.grid)
            charge = sum(self.cfg.species[s].q * self.w[s] * d for s, d in enumerate(deps))
            self.phi = poisson.solve_fe(self.grid, self._A, charge, self.cfg.kappa, self.cfg.phi_grain,
                                        self.cfg.phi_out)
            self.phi1, self.phi2 = field.nodal_gradient(self.phi, self.grid)
            return
        rho = sum(self.cfg.species[s].q * n for s, n in enumerate(self.densities(deps)))
        if self.cfg.boltzmann:
            # Boltzmann electrons: Newton from the current potential
            if self._A is None:
                self._A = poisson.assemble(self.grid)
            self.phi, _ = poisson.solve_boltzmann(self.grid, self._A, rho, self.cfg.kappa, self.cfg.phi_grain,
                                                  self.cfg.phi_out, phi0=self.phi)
        else:
            src = poisson.source_from_density(rho, self.cfg.kappa)
            self.phi = self.solver.solve(src, self.cfg.phi_grain, self.cfg.phi_out)
        self.phi1, self.phi2 = field.nodal_gradient(self.phi, self.grid)

    def set_phi(self, phi):
        self.phi = np.array(phi, dtype=np.float64)
        self.phi1, self.phi2 = field.nodal_gradient(self.phi, self.grid)

    def current_deposits(self):
        return [self.deposit(p["x1"], p["x2"]) for p in self.parts]

    def initialize_field(self):
        if not self.frozen:
            self.solve_field(self.current_deposits())

    # ------------------------------------------------------------------ move
    def _move(self, s, x1, x2, vR, vZ, vT, frac):
        """Kick (if frac is None) and drift one species; apply the boundaries.
        Returns (new arrays, keep mask)."""
        cfg, sp = self.cfg, self.cfg.species[s]
        R, Z = geo.cyl_of(x1, x2, cfg.alpha)
        qm = sp.q / sp.m
        if frac is None:
            ER, EZ = field.electric_field(self.phi1, self.phi2, x1, x2, self.grid)
            vR, vZ, vT = mover.boris_kick(vR, vZ, vT, ER, EZ, qm, cfg.kappa, cfg.wce, cfg.dt)
            step = cfg.kappa * cfg.dt
        else:
            step = cfg.kappa * cfg.dt * frac
        Rn, Zn, vRn, vZn, vTn, _, _ = mover.drift(R, Z, vR, vZ, vT, step)
        x1n, x2n = geo.conforming_of(Rn, Zn, cfg.alpha)
        hit, t_in = mover.grain_hits(R, Z, vR, vZ, vT, step, x1n, cfg.alpha)
        esc = ~hit & (x1n >= cfg.x1_out)
        if hit.any():
            h = hit
            st = step[h] if np.ndim(step) else step
            X, Y, Zi = mover.impact(R[h], Z[h], vR[h], vZ[h], vT[h], st, t_in[h], cfg.alpha)
            b, vRi, vZi, Lz = mover.impact_tallies(X, Y, Zi, vR[h], vZ[h], vT[h], self.n_bins)
            w = self.w[s]
            v2 = vR[h] ** 2 + vZ[h] ** 2 + vT[h] ** 2
            np.add.at(self.tally["count"][s], b, 1)
            np.add.at(self.tally["charge"][s], b, sp.q * w)
            np.add.at(self.tally["pR"][s], b, sp.m * w * vRi)
            np.add.at(self.tally["pZ"][s], b, sp.m * w * vZi)
            np.add.at(self.tally["L"][s], b, sp.m * w * Lz)
            np.add.at(self.tally["energy"][s], b, w * (0.5 * sp.m * v2 + sp.e_bind))
            self.absorbed[s] += int(hit.sum())
        self.escaped[s] += int(esc.sum())
        keep = ~hit & ~esc
        return (x1n, x2n, vRn, vZn, vTn), keep

    def injection_count(self, s):
        """Advance the fixed-point accumulator of species s by one step and return
        the whole number of particles to inject."""
        self.inj_acc[s] += self.inj_inc[s]
        n = self.inj_acc[s] >> 32
        self.inj_acc[s] -= n << 32
        return n

    def sample_injection(self, s, n, stream):
        """Flux-Maxwellian sample of n particles at x1_out (before the partial
        step): returns x2, vR, vZ, vT and the step fraction U."""
        cfg, sp = self.cfg, self.cfg.species[s]
        a, xo = cfg.alpha, cfg.x1_out
        slot = np.arange(n, dtype=np.uint64)
        x2 = np.zeros(n)
        todo = np.ones(n, dtype=bool)
        for k in range(MAX_ATTEMPTS):
            u0, u1, _, _ = philox4x32_10(stream, s | (P_INJ_POS << 8), slot, k, *self.key)
            cx2 = -1.0 + 2.0 * to_unit(u0)
            acc = to_unit(u1) * self.M_area <= geo.dA_dx2(xo, cx2, a)
            take = todo & (acc | (k == MAX_ATTEMPTS - 1))
            x2[take] = cx2[take]
            todo &= ~take
            if not todo.any():
                break
        u0, u1, u2, u3 = philox4x32_10(stream, s | (P_INJ_VEL << 8), slot, 0, *self.key)
        sig = np.sqrt(sp.T / sp.m)
        vn = sig * np.sqrt(-2.0 * np.log(to_unit(u0)))
        g = sig * np.sqrt(-2.0 * np.log(to_unit(u1)))
        t1 = g * np.cos(2.0 * np.pi * to_unit(u2))
        t2 = g * np.sin(2.0 * np.pi * to_unit(u2))
        x1R, x1Z, _, _ = geo.metric(np.full(n, xo), x2, a)
        gn = np.hypot(x1R, x1Z)
        nR, nZ = -x1R / gn, -x1Z / gn           # inward normal
        tR, tZ = nZ, -nR                          # in-plane tangent
        return x2, vn * nR + t1 * tR, vn * nZ + t1 * tZ, t2, to_unit(u3)

    def _inject(self, s):
        """Maxwellian-flux injection of species s at the current step."""
        n = self.injection_count(s)
        if n == 0:
            return None
        x2, vR, vZ, vT, frac = self.sample_injection(s, n, self.step_index & 0xFFFFFFFF)
        x1 = np.full(n, self.cfg.x1_out)
        ids = self.next_id[s] + np.arange(n, dtype=np.int64)
        self.next_id[s] += n
        self.injected[s] += n
        (x1n, x2n, vRn, vZn, vTn), keep = self._move(s, x1, x2, vR, vZ, vT, frac)
        return {"x1": x1n[keep], "x2": x2n[keep], "vR": vRn[keep], "vZ": vZn[keep],
                "vT": vTn[keep], "id": ids[keep]}

    def step(self):
        """One time step: push, boundaries, deposit, inject, field solve, diagnostics."""
        deps = []
        for s, p in enumerate(self.parts):
            new, keep = self._move(s, p["x1"], p["x2"], p["vR"], p["vZ"], p["vT"], None)
            self.parts[s] = {"x1": new[0][keep], "x2": new[1][keep], "vR": new[2][keep],
                             "vZ": new[3][keep], "vT": new[4][keep], "id": p["id"][keep]}
        for s in range(len(self.parts)):
            if self.inject_enabled:
                add = self._inject(s)
                if add is not None:
                    self.parts[s] = {k: np.concatenate([self.parts[s][k], add[k]]) for k in add}
            deps.append(self.deposit(self.parts[s]["x1"], self.parts[s]["x2"]))
        if not self.frozen:
            self.solve_field(deps)
        self.F_el_sum += self.electric_force()
        self.diag_steps += 1
        self.step_index += 1
        return deps

    def run(self, n_steps):
        for _ in range(n_steps):
            self.step()

    # ------------------------------------------------------------------ diagnostics
    def surface_field(self):
        """Normal field E_n = -|grad x1| dphi/dx1 at the grain nodes (i1 = 0),
        which is also the surface charge density in units of eps0 Te/(e R0)."""
        g = self.grid
        x2 = g.x2_nodes()
        x1R, x1Z, _, _ = geo.metric(np.full_like(x2, -1.0), x2, g.alpha)
        gn = np.hypot(x1R, x1Z)
        return -gn * self.phi1[:, 0], x1Z / gn

    def electric_force(self):
        """F_Z = integral over the grain of E_n^2 / 2 * n_Z dA (units eps0 Te^2/e^2),
        trapezoid rule over the grain nodes."""
        En, nZ = self.surface_field()
        g = self.grid
        x2 = g.x2_nodes()
        f = 0.5 * En * En * nZ * geo.dA_dx2(-1.0, x2, g.alpha)
        return float(np.sum(0.5 * (f[1:] + f[:-1])) * g.h2)

    def grain_charge(self):
        En, _ = self.surface_field()
        g = self.grid
        x2 = g.x2_nodes()
        f = En * geo.dA_dx2(-1.0, x2, g.alpha)
        return float(np.sum(0.5 * (f[1:] + f[:-1])) * g.h2)
