"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds parameters and random-number recipes only -- none of the method's
arithmetic.  The workloads restate the grain/plasma configurations the loop is
measured on (the paper itself gives no run sizes; see the design notes):

  c1  spherical grain, alpha = 0, B = 0, 64 x 64 cells, x1 in [-1, -0.1],
      electrons + ions with mi/me = 100, Te = Ti, lambda_D/R0 = 2,
      phi_grain = -2.5, phi_out = 0, 1e5 macro-particles per species, 200 steps,
      dt = 0.05 / omega_pe;
  c2  alpha = 0.15, B = 0, 256 x 256, hydrogen mi/me = 1836, Te = Ti,
      lambda_D/R0 = 1, 1e7 per species, 5000 steps;
  c3  alpha = 0.2, omega_ce/omega_pe = 1, 512 x 512, mi/me = 1836, Ti/Te = 0.5,
      lambda_D/R0 = 1, 5e7 per species, 2000 steps;
  c5  alpha = 0.2, omega_ce/omega_pe = 2, 2048 x 1024, x1_out = -0.02,
      mi/me = 1836, Te = Ti, lambda_D/R0 = 5, 2e8 per species, 1000 steps;
  c4  an ensemble of 64 grains (ensemble_c4): alpha uniform in [0, 0.2],
      omega_ce/omega_pe in {0, 0.5, 1}, lambda_D/R0 uniform in [0.5, 5], grids
      128 x 128, 256 x 128, 256 x 256 or 512 x 256, 1e6 - 2e7 macro-particles
      per species (log-uniform), mi/me = 1836, Te = Ti, x1_out = -0.1, 1000 steps.
"""
import numpy as np

WORKLOADS = {
    "c1": dict(alpha=0.0, wce=0.0, n1=64, n2=64, x1_out=-0.1, kappa=2.0, mi=100.0, Ti=1.0,
               n_macro=100_000, steps=200, dt=0.05, seed=0),
    "c2": dict(alpha=0.15, wce=0.0, n1=256, n2=256, x1_out=-0.1, kappa=1.0, mi=1836.0, Ti=1.0,
               n_macro=10_000_000, steps=5000, dt=0.05, seed=0),
    "c3": dict(alpha=0.2, wce=1.0, n1=512, n2=512, x1_out=-0.1, kappa=1.0, mi=1836.0, Ti=0.5,
               n_macro=50_000_000, steps=2000, dt=0.05, seed=0),
    "c5": dict(alpha=0.2, wce=2.0, n1=2048, n2=1024, x1_out=-0.02, kappa=5.0, mi=1836.0, Ti=1.0,
               n_macro=200_000_000, steps=1000, dt=0.05, seed=0),
}

C4_GRIDS = [(128, 128), (256, 128), (256, 256), (512, 256)]


def ensemble_c4(n_grains=64, particle_scale=1.0, seed=0):
    """The grains of the c4 ensemble, drawn from a seeded generator; particle
    counts can be scaled down (particle_scale < 1) for tests."""
    rng = np.random.default_rng(seed)
    out = []
    for g in range(n_grains):
        n1, n2 = C4_GRIDS[int(rng.integers(0, len(C4_GRIDS)))]
        n = float(np.exp(rng.uniform(np.log(1e6), np.log(2e7))))
        out.append(dict(alpha=float(rng.uniform(0.0, 0.2)), wce=float(rng.choice([0.0, 0.5, 1.0])),
                        n1=n1, n2=n2, x1_out=-0.1, kappa=float(rng.uniform(0.5, 5.0)), mi=1836.0, Ti=1.0,
                        n_macro=max(1, int(n * particle_scale)), steps=1000, dt=0.05, seed=0))
    return out


PHI_GRAIN = -2.5
PHI_OUT = 0.0


def scaled(name, n_macro=None, n1=None, n2=None):
    """A workload with a different particle count or grid (same physics)."""
    w = dict(WORKLOADS[name])
    if n_macro is not None:
        w["n_macro"] = int(n_macro)
    if n1 is not None:
        w["n1"] = int(n1)
    if n2 is not None:
        w["n2"] = int(n2)
    return w


def random_particles(n, x1_out, seed, v_sigma=1.0, margin=1e-3):
    """n particles uniform in the logical box (-1, x1_out) x (-1, 1) (x1 kept
    `margin` away from both boundaries) with normal velocity components."""
    rng = np.random.default_rng(seed)
    x1 = rng.uniform(-1.0 + margin, x1_out - margin, n)
    x2 = rng.uniform(-1.0, 1.0, n)
    v = rng.normal(0.0, v_sigma, (3, n))
    return x1, x2, v[0], v[1], v[2]


def smooth_density(n1, n2, seed, amplitude=1.0):
    """A smooth random charge density on the (n2+1) x (n1+1) nodes: a few
    random low-order cosine modes in the logical coordinates plus a constant."""
    rng = np.random.default_rng(seed)
    u = np.linspace(0.0, 1.0, n1 + 1)[None, :]
    v = np.linspace(0.0, 1.0, n2 + 1)[:, None]
    rho = np.full((n2 + 1, n1 + 1), 0.1 * rng.normal())
    for _ in range(6):
        a, b = rng.integers(0, 4, 2)
        rho = rho + rng.normal() * np.cos(np.pi * a * u + rng.uniform(0, np.pi)) * np.cos(
            np.pi * b * v + rng.uniform(0, np.pi))
    return amplitude * rho
