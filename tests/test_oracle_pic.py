"""Pins of the oracle's weighting, loading, injection, bookkeeping and of the
whole loop against closed-form plasma physics (Sections 1-2 of the paper)."""
import numpy as np
import pytest
from scipy import stats

from oracle import geometry as geo
from oracle.grid import Grid, node_volumes
from oracle.pic import Config, Simulation, Species


def test_deposit_partition_of_unity_and_linear_moments():
    """Bilinear weights sum to one per particle and reproduce linear functions:
    sum(dep) = N, sum(dep x1_node) = sum(x1_p), sum(dep x2_node) = sum(x2_p)."""
    cfg = Config(alpha=0.1, n1=20, n2=24, species=[Species(q=-1, m=1, n_macro=1000)])
    sim = Simulation(cfg)
    rng = np.random.default_rng(7)
    x1 = rng.uniform(-1.0, -0.1, 5000)
    x2 = rng.uniform(-1.0, 1.0, 5000)
    dep = sim.deposit(x1, x2)
    X1, X2 = sim.grid.mesh()
    assert np.isclose(dep.sum(), 5000, rtol=1e-14)
    assert np.isclose((dep * X1).sum(), x1.sum(), rtol=1e-12)
    assert np.isclose((dep * X2).sum(), x2.sum(), rtol=1e-12, atol=1e-9)
    # a particle on a node puts all its weight there
    d1 = sim.deposit(np.array([-1.0 + 3 * sim.grid.h1]), np.array([-1.0 + 5 * sim.grid.h2]))
    assert np.isclose(d1[5, 3], 1.0) and np.isclose(d1.sum(), 1.0)


@pytest.mark.parametrize("alpha", [0.0, 0.2])
def test_uniform_load_gives_unit_density(alpha):
    """A load uniform in physical volume, weighted with V_ij = integral hat dOmega,
    has expected density n0 at every node; per-node deviations are within the
    Poisson noise (the variance of a sum of hats is at most its mean)."""
    N = 400000
    cfg = Config(alpha=alpha, n1=12, n2=10, x1_out=-0.4, seed=11,
                 species=[Species(q=-1, m=1, n_macro=N)])
    sim = Simulation(cfg)
    sim.load(0)
    dep = sim.deposit(sim.parts[0]["x1"], sim.parts[0]["x2"])
    expect = N * sim.vol / sim.V
    z = (dep - expect) / np.sqrt(expect)
    assert np.mean(z * z) < 1.3
    assert np.max(np.abs(z)) < 5.0
    n = sim.densities([dep])[0]
    big = expect > 2000
    assert np.all(np.abs(n[big] - 1.0) < 5.0 / np.sqrt(expect[big]))


def test_load_velocities_are_maxwellian():
    cfg = Config(alpha=0.1, n1=8, n2=8, seed=3, species=[Species(q=1, m=4.0, T=0.5, n_macro=200000)])
    sim = Simulation(cfg)
    sim.load(0)
    sig = np.sqrt(0.5 / 4.0)
    for k in ("vR", "vZ", "vT"):
        v = sim.parts[0][k] / sig
        assert stats.kstest(v, "norm").pvalue > 1e-3


def test_injection_count_closed_form():
    """alpha = 0: A_out = 4 pi r_out^2 and the per-step count is
    n sqrt(T/(2 pi m)) A_out kappa dt / w; the fixed-point accumulator delivers
    floor(k N) particles after k steps (exact integers)."""
    w = 0.013
    cfg = Config(alpha=0.0, n1=8, n2=8, x1_out=-0.25, kappa=1.7, dt=0.03,
                 species=[Species(q=1, m=9.0, T=0.7, weight=w)])
    sim = Simulation(cfg)
    n_real = np.sqrt(0.7 / (2 * np.pi * 9.0)) * 4 * np.pi * 16.0 * 1.7 * 0.03 / w
    total = sum(sim.injection_count(0) for _ in range(1000))
    assert abs(total - np.floor(1000 * n_real)) <= 1


@pytest.mark.parametrize("alpha", [0.0, 0.2])
def test_injection_sample_is_a_flux_maxwellian(alpha):
    """Injected x2 has density proportional to eq. (4) at x1_out; the inward
    normal velocity is Rayleigh (the flux-weighted half-Maxwellian), the two
    tangential components are normal with variance T/m."""
    T, m = 2.0, 3.0
    cfg = Config(alpha=alpha, n1=8, n2=8, x1_out=-0.3, seed=5, species=[Species(q=1, m=m, T=T, weight=1.0)])
    sim = Simulation(cfg)
    n = 200000
    x2, vR, vZ, vT, frac = sim.sample_injection(0, n, 17)
    sig = np.sqrt(T / m)
    x1R, x1Z, _, _ = geo.metric(np.full(n, -0.3), x2, alpha)
    g = np.hypot(x1R, x1Z)
    vn = -(vR * x1R + vZ * x1Z) / g
    vt = (vR * x1Z - vZ * x1R) / g
    assert np.all(vn > 0)
    assert stats.kstest(vn / sig, "rayleigh").pvalue > 1e-3
    assert stats.kstest(vt / sig, "norm").pvalue > 1e-3
    assert stats.kstest(vT / sig, "norm").pvalue > 1e-3
    assert stats.kstest(frac, "uniform").pvalue > 1e-3
    # x2 against the normalised cumulative of eq. (4)
    grid = np.linspace(-1, 1, 4001)
    pdf = geo.dA_dx2(-0.3, grid, alpha)
    cdf = np.concatenate([[0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
    cdf /= cdf[-1]
    assert stats.kstest(x2, lambda t: np.interp(t, grid, cdf)).pvalue > 1e-3
    if alpha == 0.0:
        assert stats.kstest(x2, "uniform", args=(-1, 2)).pvalue > 1e-3


def test_particle_bookkeeping_is_exact():
    """injected + loaded = absorbed + escaped + resident, exact integers, in a
    self-consistent run with both species and an axial field."""
    cfg = Config(alpha=0.15, n1=16, n2=16, wce=0.8, kappa=2.0, seed=2,
                 species=[Species(q=-1, m=1, n_macro=20000), Species(q=1, m=25, n_macro=20000)])
    sim = Simulation(cfg)
    sim.load(0)
    sim.load(1)
    sim.initialize_field()
    sim.run(25)
    for s in range(2):
        assert 20000 + sim.injected[s] == sim.absorbed[s] + sim.escaped[s] + sim.resident(s)
        assert sim.tally["count"][s].sum() == sim.absorbed[s]
        ids = sim.parts[s]["id"]
        assert len(np.unique(ids)) == len(ids)
    assert sim.injected[0] > 0 and sim.absorbed[0] > 0 and sim.escaped[0] > 0


@pytest.mark.slow
def test_repelled_electron_current_to_a_sphere_is_boltzmann():
    """alpha = 0, B = 0, a monotonic repelling potential (the vacuum solution,
    frozen), Maxwellian flux injected at r_out: every trajectory reaching the
    sphere comes from the source, so by Liouville the collected flux is the
    thermal flux times exp(-e |phi_g| / Te):  I = 4 pi R0^2 n0 sqrt(Te/2 pi me)
    exp(e phi_g / Te).  Also the spherical grain feels no net momentum
    (no force, Section 3) and no torque, and the impact tallies mirror in x2."""
    w = 5.0e-4
    cfg = Config(alpha=0.0, n1=32, n2=32, x1_out=-0.5, kappa=1.0, dt=0.05, seed=9,
                 phi_grain=-2.5, species=[Species(q=-1, m=1, T=1, weight=w)])
    sim = Simulation(cfg)
    X1, _ = sim.grid.mesh()
    sim.set_phi(-2.5 + 2.5 * (X1 + 1.0) / 0.5)
    sim.frozen = True
    sim.run(60)
    a0 = sim.absorbed[0]
    counts0 = sim.tally["count"][0].copy()
    pz0, L0 = sim.tally["pZ"][0].copy(), sim.tally["L"][0].copy()
    n_meas = 150
    sim.run(n_meas)
    absorbed = sim.absorbed[0] - a0
    expect = np.sqrt(1 / (2 * np.pi)) * np.exp(-2.5) * 4 * np.pi * 1.0 * cfg.dt * n_meas / w
    sigma = np.sqrt(expect)
    assert abs(absorbed - expect) < 4 * sigma + 0.02 * expect, (absorbed, expect)
    c = sim.tally["count"][0] - counts0
    half = len(c) // 2
    lo, hi = c[:half].sum(), c[half:].sum()
    assert abs(lo - hi) < 4 * np.sqrt(lo + hi)
    pz = sim.tally["pZ"][0] - pz0
    L = sim.tally["L"][0] - L0
    # per-particle |p_Z| and |L| are O(1); the sums of N random-sign terms are O(sqrt N)
    assert abs(pz.sum()) < 4 * np.sqrt(absorbed) * w * 2.0
    assert abs(L.sum()) < 4 * np.sqrt(absorbed) * w * 2.0
