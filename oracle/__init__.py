"""Plain FP64 CPU oracle of the aspherical PIC method (arXiv 2307.11107).

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg of
the benchmark may import it.  The product path (the HIP library and its Python
binding) never imports, calls or links anything here, and shares no code with it.

Modules: philox (random numbers), geometry (eqs. 1-5, 7, 8, 10), grid (uniform
(x1, x2) grid, node volumes), poisson (eqs. 6-7 by LU), field (eq. 10, gradient
and interpolation), mover (eq. 9, leapfrog, boundaries), pic (the time loop,
loading, injection, tallies, grain diagnostics).

Parity unpinned: the multi-step self-consistent tallies of `pic.Simulation`
beyond the closed forms the tests check (Boltzmann-attenuated electron current
to a sphere, the spherical-grain symmetry, particle bookkeeping) -- a plasma
simulation has no closed-form end state.
"""
