"""Particle mover of eq. (9) and the grain / outer-boundary treatment, FP64.

Oracle module (test infrastructure only; the product path never imports it).

Paper passages:
  * Section 2, eq. (9): motion in cylindrical (R, Z) with velocity components
    (V_R, V_Z, V_Theta), the electric force, the axial-field Lorentz terms
    -V_Theta B (in dV_R/dt) and +V_R B (in dV_Theta/dt), the centrifugal term
    V_Theta^2 / R and the Coriolis term -V_R V_Theta / R;
  * Section 2: eq. (9) is advanced with an explicit leapfrog scheme;
  * Section 1: particles reaching the grain give it their charge, momentum,
    angular momentum and energy at the point of impact; particles may leave
    through the outer boundary.

Readings (see also the module docstring of `pic`):
  * units: lengths in R0, time in 1/omega_pe, velocity in v_te = sqrt(Te/me),
    E in Te/(e R0).  Then dv/dt = (q/m) kappa E, dx/dt = kappa v with
    kappa = lambda_D / R0, and the field term of eq. (9) turns velocities at the
    rate omega = (q/m) (omega_ce/omega_pe)  (q in e, m in me);
  * leapfrog: positions at integer steps, velocities at half steps.  The kick is
    the Boris form (half electric kick, exact-angle rotation of (V_R, V_Theta) by
    2 atan(omega dt / 2) in the sense eq. (9) fixes, half electric kick).  The
    drift is a straight line in the local Cartesian frame (R-hat, Theta-hat,
    Z-hat) followed by a rotation of (V_R, V_Theta) into the meridional plane of
    the new position; this carries the centrifugal and Coriolis terms of eq. (9)
    exactly and has no singularity on the axis.  As dt -> 0 it converges to
    eq. (9) (pinned against an ODE integration of eq. (9) in the tests);
  * a particle is absorbed when the new position has x1 <= -1 or when the
    straight chord of the step has x1 <= -1 at its point of closest approach to
    the origin; the impact point is then found by bisection on x1 + 1 along the
    chord.  A particle whose new position has x1 >= x1_out escapes.
"""
import numpy as np

from . import geometry as geo

BISECTION_STEPS = 48


def boris_kick(vR, vZ, vT, ER, EZ, qm, kappa, wce, dt):
    """Kick v^{n-1/2} -> v^{n+1/2} with E at x^n (eq. 9, velocity equations
    without the inertial terms, which the drift applies)."""
    a = 0.5 * qm * kappa * dt
    vR = vR + a * ER
    vZ = vZ + a * EZ
    if wce != 0.0:
        t = 0.5 * qm * wce * dt
        c = (1.0 - t * t) / (1.0 + t * t)
        s = 2.0 * t / (1.0 + t * t)
        # dV_R/dt = -omega V_Theta, dV_Theta/dt = +omega V_R  (eq. 9)
        vR, vT = c * vR - s * vT, s * vR + c * vT
    vR = vR + a * ER
    vZ = vZ + a * EZ
    return vR, vZ, vT


def drift(R, Z, vR, vZ, vT, step):
    """Straight-line move by `step` * v in the local Cartesian frame, then the
    rotation of (v_R, v_Theta) into the meridional plane of the new point.
    Returns (R', Z', vR', vZ, vT', X, Y) with (X, Y) the Cartesian endpoint."""
    X = R + step * vR
    Y = step * vT
    Rn = np.hypot(X, Y)
    safe = Rn > 0.0
    c = np.where(safe, X / np.where(safe, Rn, 1.0), 1.0)
    s = np.where(safe, Y / np.where(safe, Rn, 1.0), 0.0)
    return Rn, Z + step * vZ, c * vR + s * vT, vZ, -s * vR + c * vT, X, Y


def _x1_on_chord(R0, Z0, dX, dY, dZ, t, alpha):
    X = R0 + t * dX
    Y = t * dY
    Z = Z0 + t * dZ
    x1, _ = geo.conforming_of(np.hypot(X, Y), Z, alpha)
    return x1


def grain_hits(R, Z, vR, vZ, vT, step, x1_new, alpha):
    """Absorption test.  Returns (hit mask, t_in) where t_in in (0, 1] is a chord
    parameter known to be inside the grain for the hits."""
    dX, dY, dZ = step * vR, step * vT, step * vZ
    dd = dX * dX + dY * dY + dZ * dZ
    tc = np.where(dd > 0.0, -(R * dX + Z * dZ) / np.where(dd > 0.0, dd, 1.0), 0.0)
    tc = np.clip(tc, 0.0, 1.0)
    x1c = _x1_on_chord(R, Z, dX, dY, dZ, tc, alpha)
    # "not outside" rather than "x1 <= -1": the origin, where x1 is undefined,
    # lies inside the grain
    end_in = ~(x1_new > -1.0)
    mid_in = ~(x1c > -1.0)
    hit = end_in | mid_in
    t_in = np.where(mid_in, tc, 1.0)
    return hit, t_in


def impact(R, Z, vR, vZ, vT, step, t_in, alpha):
    """Bisection on x1 + 1 along the chord between t = 0 (outside) and t_in
    (inside).  Returns the Cartesian impact point (X, Y, Z)."""
    dX, dY, dZ = step * vR, step * vT, step * vZ
    lo = np.zeros_like(t_in)
    hi = np.array(t_in, dtype=np.float64, copy=True)
    for _ in range(BISECTION_STEPS):
        mid = 0.5 * (lo + hi)
        inside = ~(_x1_on_chord(R, Z, dX, dY, dZ, mid, alpha) > -1.0)
        hi = np.where(inside, mid, hi)
        lo = np.where(inside, lo, mid)
    t = hi
    return R + t * dX, t * dY, Z + t * dZ


def impact_tallies(X, Y, Zi, vR, vZ, vT, n_bins):
    """Bin of the impact (by x2 = cos(theta) of the impact point, n_bins equal
    bins over [-1, 1]) and the momentum / angular momentum carried in, per unit
    mass.  v is the Cartesian velocity (vR, vT, vZ) in the frame of the start
    point; it is rotated into the meridional plane of the impact point."""
    Ri = np.hypot(X, Y)
    r = np.hypot(Ri, Zi)
    x2 = Zi / r
    b = np.clip(np.floor((x2 + 1.0) * 0.5 * n_bins).astype(np.int64), 0, n_bins - 1)
    safe = Ri > 0.0
    c = np.where(safe, X / np.where(safe, Ri, 1.0), 1.0)
    s = np.where(safe, Y / np.where(safe, Ri, 1.0), 0.0)
    vRi = c * vR + s * vT
    vTi = -s * vR + c * vT
    return b, vRi, vZ, Ri * vTi
