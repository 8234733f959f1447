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
  * a particle is absorbed when the straight chord of its step meets the grain
    (Section 1: particles intersecting the grain are absorbed), and the impact
    point is the chord's first point on the grain surface.  The grain is the
    region r <= rho(x2) around the origin bounded by x1 = -1, with
    rho(x2) = (1 + sqrt(1 + 4 alpha x2)) / 2 from eq. (3).  Eq. (2)'s
    x1 <= -1, multiplied by r^3, reads G = r^3 - r^2 - alpha Z <= 0: it holds
    on the shell r_low(x2) <= r <= rho(x2) between the two roots of
    r^2 - r - alpha x2, and the core r < r_low next to the origin (where x1 of
    eq. 2 is not below -1) is reached only through that shell, so the chord's
    first point with G <= 0 is its first point on the grain.  The test is exact
    (up to rounding) for any |alpha| < 1/4: along a chord G is convex except
    on one stretch around the closest approach to the origin where it is
    concave (see chord_impact), so the first point with G <= 0 is found piece
    by piece.  A particle whose new position has x1 >= x1_out escapes.
"""
import numpy as np

from . import geometry as geo

BISECTION_STEPS = 60


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


def _chord_G(a, b, c, Z0, dZ, t, alpha):
    """G = r^3 - r^2 - alpha Z and dG/dt at parameter t of the chord
    P(t) = P0 + t d, with a = |d|^2, b = P0.d, c = |P0|^2 (r^2 = c + 2bt + at^2)."""
    q = c + t * (2.0 * b + a * t)
    r = np.sqrt(np.maximum(q, 0.0))
    G = r * q - q - alpha * (Z0 + t * dZ)
    dG = (3.0 * r - 2.0) * (b + a * t) - alpha * dZ
    return G, dG


def chord_impact(R, Z, dX, dY, dZ, alpha):
    """First point of the chord P(t) = (R + t dX, t dY, Z + t dZ), t in [0, 1],
    inside the grain.  Returns (hit mask, t of the first crossing).

    Along the chord, with t* the parameter and r* the distance of the closest
    approach to the origin, d2G/dt2 = |d|^2 (6 r^2 - 2 r - 3 r*^2) / r, negative
    only where r < r_c = (1 + sqrt(1 + 18 r*^2)) / 6 (possible only if
    r* < 2/3): G is convex on t <= t* - s_c, concave on |t - t*| <= s_c and
    convex on t >= t* + s_c (s_c = 0 if r* >= 2/3).  A convex piece's minimum
    is at the root of dG/dt (bisection), a concave piece's at an end point.  The
    pieces are searched in order; in the first whose minimum is <= 0 the
    crossing is unique (G falls monotonically to that minimum on a convex
    piece; a concave piece positive at its start changes sign once) and is
    found by bisection on G.  Only the part of the chord inside r <= rho_max
    (the largest grain radius) can meet the grain."""
    R, Z, dX, dY, dZ = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (R, Z, dX, dY, dZ)))
    shape = R.shape
    R, Z, dX, dY, dZ = (v.ravel() for v in (R, Z, dX, dY, dZ))
    rho_max = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * abs(alpha)))
    a = dX * dX + dY * dY + dZ * dZ
    b = R * dX + Z * dZ
    c = R * R + Z * Z
    moving = a > 0.0
    aa = np.where(moving, a, 1.0)
    disc = b * b - aa * (c - rho_max * rho_max)
    sq = np.sqrt(np.maximum(disc, 0.0))
    lo = np.maximum(0.0, (-b - sq) / aa)
    hi = np.minimum(1.0, (-b + sq) / aa)
    # the chords that enter r <= rho_max; the others miss the grain
    cand = moving & (disc >= 0.0) & (lo <= hi)
    hit_all = np.zeros(R.shape, dtype=bool)
    t_all = np.zeros(R.shape)
    k = np.nonzero(cand)[0]
    if k.size == 0:
        return hit_all.reshape(shape), t_all.reshape(shape)
    aa, b, c, Z, dZ, lo, hi = aa[k], b[k], c[k], Z[k], dZ[k], lo[k], hi[k]
    cand = np.ones(k.size, dtype=bool)
    ts = -b / aa
    rs2 = np.maximum(c - b * b / aa, 0.0)
    rc = (1.0 + np.sqrt(1.0 + 18.0 * rs2)) / 6.0
    sc = np.where(rs2 < 4.0 / 9.0, np.sqrt(np.maximum(rc * rc - rs2, 0.0) / aa), 0.0)
    G = lambda t: _chord_G(aa, b, c, Z, dZ, t, alpha)[0]
    dG = lambda t: _chord_G(aa, b, c, Z, dZ, t, alpha)[1]
    found = np.zeros(k.size, dtype=bool)
    t_out = np.zeros(k.size)
    t_in = np.zeros(k.size)
    pieces = ((lo, np.minimum(hi, ts - sc), True),
              (np.maximum(lo, ts - sc), np.minimum(hi, ts + sc), False),
              (np.maximum(lo, ts + sc), hi, True))
    for left, right, convex in pieces:
        todo = cand & ~found & (left <= right)
        if not todo.any():
            continue
        if convex:
            # minimum of a convex piece: where dG/dt changes sign
            u, v = left.copy(), right.copy()
            for _ in range(BISECTION_STEPS):
                m = 0.5 * (u + v)
                up = dG(m) >= 0.0
                v = np.where(up, m, v)
                u = np.where(up, u, m)
            tm = np.where(dG(left) >= 0.0, left, np.where(dG(right) <= 0.0, right, v))
        else:
            tm = np.where(G(left) <= G(right), left, right)
        new = todo & (G(tm) <= 0.0)
        t_out = np.where(new, left, t_out)
        t_in = np.where(new, tm, t_in)
        found |= new
    # first crossing: bisection on G between an outside and an inside point
    u, v = t_out.copy(), t_in.copy()
    for _ in range(BISECTION_STEPS):
        m = 0.5 * (u + v)
        inside = G(m) <= 0.0
        v = np.where(inside, m, v)
        u = np.where(inside, u, m)
    t_hit = np.where(G(t_out) <= 0.0, t_out, v)
    hit_all[k] = found
    t_all[k] = np.where(found, t_hit, 0.0)
    return hit_all.reshape(shape), t_all.reshape(shape)


def grain_hits(R, Z, vR, vZ, vT, step, x1_new, alpha):
    """Absorption test of a step.  Returns (hit mask, t of the impact point on
    the chord).  An end point with x1 <= -1 that the chord test missed by
    rounding (a grazing end point) is absorbed there."""
    hit, t = chord_impact(R, Z, step * vR, step * vT, step * vZ, alpha)
    end_in = ~(x1_new > -1.0)
    return hit | end_in, np.where(hit, t, 1.0)


def impact(R, Z, vR, vZ, vT, step, t, alpha):
    """The Cartesian point (X, Y, Z) at parameter t of the step's chord."""
    return R + t * step * vR, t * step * vT, Z + t * step * vZ


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
