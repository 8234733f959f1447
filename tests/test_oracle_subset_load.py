"""The oracle's load of a subset of indices draws exactly the particles of the
full load with those indices (Philox counters depend on the index alone)."""
import numpy as np

from oracle.pic import Config, Simulation, Species


def test_subset_load_equals_full_load():
    cfg = Config(alpha=0.2, n1=32, n2=32, x1_out=-0.1, wce=1.0, kappa=1.0, dt=0.05, seed=3,
                 species=[Species(q=-1.0, m=1.0, n_macro=5000), Species(q=1.0, m=1836.0, T=0.5, n_macro=5000)])
    full = Simulation(cfg)
    part = Simulation(cfg)
    ids = np.array([0, 7, 123, 4999, 2500, 42])
    for s in range(2):
        full.load(s)
        part.load(s, slots=ids)
        a = full.particles(s)
        b = part.particles(s)
        order = np.sort(ids)
        assert np.array_equal(b["id"], order)
        for k in ("x1", "x2", "vR", "vZ", "vT"):
            assert np.array_equal(a[k][order], b[k])
