// Particle kernels of the aspherical PIC loop for gfx950.
//
// One step of a particle (paper, Section 2): the nodal (dphi/dx1, dphi/dx2) are
// interpolated bilinearly to the particle and combined with the analytic
// coordinate derivatives into (E_R, E_Z) (eq. 10); eq. (9) is advanced by a
// leapfrog step -- Boris kick with the axial-field rotation, straight drift in
// the local Cartesian frame and rotation of (v_R, v_Theta) into the new
// meridional plane, which carries the centrifugal and Coriolis terms of eq. (9);
// particles whose new position or whose chord lies inside the grain (x1 <= -1)
// are absorbed and tallied per x2-bin of the impact point (Section 1: charge,
// momentum, angular momentum, energy transferred at the point of impact);
// particles beyond x1_out escape; the others deposit their charge with
// bilinear weights (the volume element of eq. (5) enters through the node
// volumes when the density is formed).
//
// Two storage forms:
//   FP32 split  -- int32 packed cell (i2 << 16 | i1), float offsets f1, f2 in
//                  [0,1), float velocities: 24 bytes per particle.  The new
//                  position is formed from the displacement (differences of
//                  eqs. 2-3), never by recomputing x1 from (R, Z), so position
//                  resolution is ~1e-7 of a cell everywhere, also next to the
//                  grain and the axis.
//   FP64 plain  -- double x1, x2 and velocities: 40 bytes per particle.
// Dead slots: packed cell < 0 (FP32) or x1 > 0 (FP64); they are removed by the
// periodic counting sort.
// Multiply-adds are fused only within one source expression, never across
// statements: the push loop inlines the particle update twice (two particles
// per iteration), and both copies must round alike so that a particle's
// trajectory does not depend on the slot it occupies.
#pragma clang fp contract(on)

#include "apic_internal.h"
#include "device_common.h"

#include <algorithm>
#include <mutex>
#include <type_traits>

namespace apic {

constexpr int BLOCK = 256;
// Largest workgroup of the persistent push and deposit kernels (their sizes
// are PushTraits<SPLIT>::NT).
constexpr int PUSH_BLOCK_MAX = 512;
constexpr double FP64_DEAD = 1.0;   // x1 of a dead FP64 slot (valid x1 < 0)

__device__ inline void atomic_add_f64(double* p, double v) { gadd(p, v); }

// Block-wide sum of a per-thread u32 followed by one atomic per block.
__device__ inline void block_count_add(uint32_t v, unsigned long long* dst) {
    __shared__ uint32_t red[(BLOCK > PUSH_BLOCK_MAX ? BLOCK : PUSH_BLOCK_MAX) / 64];
    uint32_t w = v;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
        if (t) gadd(dst, (unsigned long long)t);
    }
    __syncthreads();
}

// ----------------------------------------------------------------- grain impact
// The chord of a step, P(t) = (R + t dX, t dY, Z + t dZ) for t in [0, 1], meets
// the grain where eq. (2)'s x1 <= -1, multiplied by r^3, holds:
// G = r^3 - r^2 - alpha Z <= 0.  That is the shell between the two roots of
// r^2 - r - alpha x2, whose outer root is the grain radius of eq. (3); the core
// next to the origin (where x1 of eq. 2 is not below -1) is reached only
// through the shell, so the chord's first point with G <= 0 is its first point
// on the grain.  With r^2 = c + 2 b t + a t^2 (a = |d|^2, b = P0.d,
// c = |P0|^2) and r* the chord's closest distance to the origin,
// d2G/dt2 = a (6 r^2 - 2 r - 3 r*^2) / r: G is concave where
// r < r_c = (1 + sqrt(1 + 18 r*^2)) / 6 (only if r* < 2/3) and convex elsewhere,
// so the chord falls into at most three pieces -- convex, concave, convex.
template <typename T>
struct Chord {
    T a, b, c, Z, dZ, alpha;
    __device__ T G(T t) const {
        const T q = c + t * (T(2) * b + a * t);
        const T r = sqrt(q > T(0) ? q : T(0));
        return r * q - q - alpha * (Z + t * dZ);
    }
    __device__ T dG(T t) const {
        const T q = c + t * (T(2) * b + a * t);
        const T r = sqrt(q > T(0) ? q : T(0));
        return (T(3) * r - T(2)) * (b + a * t) - alpha * dZ;
    }
};

// t of the chord's first point inside the grain, or -1 if the chord misses it.
// Only the part within r <= rho_max (the largest grain radius) is searched.
// The pieces are taken in order: a convex piece's minimum is the root of dG/dt
// (bisection), a concave piece's lies at an end; in the first piece whose
// minimum is <= 0 the crossing is unique (G falls monotonically to a convex
// minimum; a concave piece positive at its start changes sign once) and is
// found by bisection on G.
template <typename T>
__device__ __attribute__((noinline)) T chord_hit(T rho_max, T alpha, T R, T Z, T dX, T dY, T dZ, int iters) {
    const Chord<T> ch{dX * dX + dY * dY + dZ * dZ, R * dX + Z * dZ, R * R + Z * Z, Z, dZ, alpha};
    if (!(ch.a > T(0))) return T(-1);
    const T disc = ch.b * ch.b - ch.a * (ch.c - rho_max * rho_max);
    if (!(disc >= T(0))) return T(-1);
    const T sq = sqrt(disc);
    const T lo = max(T(0), (-ch.b - sq) / ch.a), hi = min(T(1), (-ch.b + sq) / ch.a);
    if (!(lo <= hi)) return T(-1);
    const T ts = -ch.b / ch.a;
    const T rs2 = max(T(0), ch.c - ch.b * ch.b / ch.a);
    T sc = T(0);
    if (rs2 < T(4) / T(9)) {
        const T rc = (T(1) + sqrt(T(1) + T(18) * rs2)) / T(6);
        sc = sqrt(max(T(0), rc * rc - rs2) / ch.a);
    }
    for (int k = 0; k < 3; ++k) {
        const T L = k == 0 ? lo : max(lo, k == 1 ? ts - sc : ts + sc);
        const T U = k == 2 ? hi : min(hi, k == 0 ? ts - sc : ts + sc);
        if (!(L <= U)) continue;
        T tm;
        if (k == 1) {
            tm = ch.G(L) <= ch.G(U) ? L : U;
        } else if (ch.dG(L) >= T(0)) {
            tm = L;
        } else if (ch.dG(U) <= T(0)) {
            tm = U;
        } else {
            T u = L, v = U;
            for (int it = 0; it < iters; ++it) {
                const T m = T(0.5) * (u + v);
                const bool up = ch.dG(m) >= T(0);
                v = up ? m : v;
                u = up ? u : m;
            }
            tm = v;
        }
        if (!(ch.G(tm) <= T(0))) continue;
        if (ch.G(L) <= T(0)) return L;
        T u = L, v = tm;
        for (int it = 0; it < iters; ++it) {
            const T m = T(0.5) * (u + v);
            const bool in = ch.G(m) <= T(0);
            v = in ? m : v;
            u = in ? u : m;
        }
        return v;
    }
    return T(-1);
}

// Chord test of a step: -1 unless the chord comes within rho_max of the
// origin (the usual case, decided here without the search).  The squared
// distance of the chord's closest point, m = clamp(-P.d, 0, |d|^2) along it,
// times |d|^2 is |P|^2 |d|^2 - m (2 (-P.d) - m): no division.
template <typename T>
__device__ inline T grain_chord(T rho_max, T alpha, T R, T Z, T dX, T dY, T dZ, int iters) {
    const T dd = dX * dX + dY * dY + dZ * dZ;
    const T pd = -(R * dX + Z * dZ);
    const T m = pd > T(0) ? (pd < dd ? pd : dd) : T(0);
    const T c = R * R + Z * Z;
    if (c * dd - m * (T(2) * pd - m) > rho_max * rho_max * dd) return T(-1);
    return chord_hit<T>(rho_max, alpha, R, Z, dX, dY, dZ, iters);
}

// Tallies of an absorbed particle at the chord's impact point t: the velocity
// is rotated into the impact point's meridional plane.  The impact parameters
// come as scalars (no struct by reference), so a caller's parameter structs can
// stay in registers.
struct ImpactSpecies {
    double q, m, w, e_bind;
};

template <typename T>
__device__ __attribute__((noinline)) void tally_impact(int n_bins, ImpactSpecies sp, int s, int ns,
                             T R, T Z, T dX, T dY, T dZ, T t, T vR, T vZ, T vT,
                             double* tally, unsigned long long* tally_count) {
    const T X = R + t * dX, Y = t * dY, Zi = Z + t * dZ;
    const T Ri = sqrt(X * X + Y * Y);
    const T ri = sqrt(Ri * Ri + Zi * Zi);
    const T x2 = Zi / ri;
    int b = (int)floor((x2 + T(1)) * T(0.5) * (T)n_bins);
    b = b < 0 ? 0 : (b >= n_bins ? n_bins - 1 : b);
    T c = 1, sn = 0;
    if (Ri > T(0)) { c = X / Ri; sn = Y / Ri; }
    const double vRi = (double)(c * vR + sn * vT);
    const double vTi = (double)(-sn * vR + c * vT);
    const double v2 = (double)vR * vR + (double)vZ * vZ + (double)vT * vT;
    const size_t stride = (size_t)ns * n_bins;
    const size_t o = (size_t)s * n_bins + b;
    atomic_add_f64(&tally[o], sp.q * sp.w);
    atomic_add_f64(&tally[stride + o], sp.m * sp.w * vRi);
    atomic_add_f64(&tally[2 * stride + o], sp.m * sp.w * (double)vZ);
    atomic_add_f64(&tally[3 * stride + o], sp.m * sp.w * (double)Ri * vTi);
    atomic_add_f64(&tally[4 * stride + o], sp.w * (0.5 * sp.m * v2 + sp.e_bind));
    gadd(&tally_count[o], 1ull);
}

// ----------------------------------------------------------------- FP32 split push
// Hardware reciprocal and square root (about 1 ulp) replace the correctly
// rounded FP32 division and sqrt sequences in the split kernel; the position
// update is formed from differences, so 1-ulp factors perturb a displacement
// only by ~1e-7 of itself.
__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

// One particle of the FP32 split form.  Returns -1 for a dead slot, 0 if the
// particle stays (new cell and offsets in i1n, i2n, f1n, f2n), 1 if absorbed,
// 2 if escaped; the particle's slot is updated in place.
struct SplitConsts {
    int n1, n2, nx;
    float alpha, h1, h2, ih1, ih2, mx1_out, step, qmh, rcm1, rs;
};

__device__ inline SplitConsts split_consts(const GrainParams& gp, const SpeciesParams& sp) {
    SplitConsts k;
    k.n1 = gp.n1;
    k.n2 = gp.n2;
    k.nx = gp.nx;
    k.alpha = (float)gp.alpha;
    k.h1 = (float)gp.h1;
    k.h2 = (float)gp.h2;
    k.ih1 = (float)gp.inv_h1;
    k.ih2 = (float)gp.inv_h2;
    k.mx1_out = (float)(-gp.x1_out);
    k.step = (float)gp.step;
    k.qmh = (float)sp.qm_half;
    k.rcm1 = (float)sp.rot_cm1;
    k.rs = (float)sp.rot_s;
    return k;
}

struct SplitState {
    int32_t c;
    float f1, f2, vR, vZ, vT;
    unsigned long long g[4];   // push: the float2 nodal gradients of the cell, bit patterns
};

// Slot p of a 4-byte particle array, addressed as the array base plus a
// 32-bit byte offset (a task holds fewer than 2^30 slots): the loads and
// stores then take the base from scalar registers and share one offset
// register instead of forming a 64-bit address per array.
template <typename T>
__device__ __forceinline__ gptr<T> slot4(T* base, int64_t p) {
    static_assert(sizeof(T) == 4, "4-byte elements");
    using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return (gptr<T>)((gptr<C>)gbl(reinterpret_cast<C*>(base)) + ((uint32_t)p << 2));
}

// The particle arrays stream through once per step: the push's loads and
// stores of them are non-temporal, which keeps L2 for the field and the deposit.
template <typename T>
__device__ __forceinline__ T ld_stream(gptr<const T> a) { return __builtin_nontemporal_load(a); }
template <typename T>
__device__ __forceinline__ void st_stream(gptr<T> a, T v) { __builtin_nontemporal_store(v, a); }

__device__ inline SplitState load_split(const PBuf& b, int64_t p) {
    SplitState q;
    q.c = *slot4(static_cast<const int32_t*>(b.pos0), p);
    q.f1 = *slot4(static_cast<const float*>(b.pos1), p);
    q.f2 = *slot4(static_cast<const float*>(b.pos2), p);
    q.vR = *slot4(static_cast<const float*>(b.vR), p);
    q.vZ = *slot4(static_cast<const float*>(b.vZ), p);
    q.vT = *slot4(static_cast<const float*>(b.vT), p);
    return q;
}

__device__ inline void set_dead(SplitState& q) { q.c = DEAD; }
__device__ inline bool is_dead(const SplitState& q) { return q.c < 0; }

// Advances one particle given its loaded state q; writes slot p of b.
__device__ inline int push_split_one(const GrainParams& gp, const SpeciesParams& sp,
                                     const SplitConsts& K, int s, int ns, int64_t p,
                                     const SplitState& q, const PBuf& b, double* __restrict__ tally,
                                     unsigned long long* __restrict__ tally_count, int& i1n,
                                     int& i2n, float& f1n, float& f2n) {
    const int32_t c = q.c;
    if (c < 0) return -1;
    const gptr<int32_t> cell = slot4(static_cast<int32_t*>(b.pos0), p);
    const int n1 = K.n1, n2 = K.n2, nx = K.nx;
    const float alpha = K.alpha, h1 = K.h1, h2 = K.h2, qmh = K.qmh, step = K.step;
    const int i1 = cell_i1(c), i2 = cell_i2(c);
    const float f1 = q.f1, f2 = q.f2;
    float vR = q.vR, vZ = q.vZ, vT = q.vT;

    // gather (bilinear in the logical coordinates); the cell's nodal gradients
    // were loaded with the particle's state
    const float2 g00 = __builtin_bit_cast(float2, q.g[0]), g10 = __builtin_bit_cast(float2, q.g[1]);
    const float2 g01 = __builtin_bit_cast(float2, q.g[2]), g11 = __builtin_bit_cast(float2, q.g[3]);
    const float e1 = 1.f - f1, e2 = 1.f - f2;
    const float w00 = e1 * e2, w10 = f1 * e2, w01 = e1 * f2, w11 = f1 * f2;
    const float p1 = w00 * g00.x + w10 * g10.x + w01 * g01.x + w11 * g11.x;
    const float p2 = w00 * g00.y + w10 * g10.y + w01 * g01.y + w11 * g11.y;

    // geometry at the particle from the cell index: -x1 measured from the
    // outer boundary (no cancellation where |x1| is small), 1 + x2 and 1 - x2
    // measured from the two axis ends
    const float mx1 = K.mx1_out + ((float)(n1 - i1) - f1) * h1;      // -x1 > 0
    const float opx2 = ((float)i2 + f2) * h2;
    const float omx2 = ((float)(n2 - i2) - f2) * h2;
    const float x2 = 0.5f * (opx2 - omx2);
    const float sn = fsqrt(opx2 * omx2);
    // eq. (3) with x1 = -mx1
    const float imx1 = frcp(mx1);
    const float r = 0.5f * (1.f + fsqrt(1.f + 4.f * alpha * mx1 * x2)) * imx1;
    const float R = r * sn, Z = r * x2;
    // analytic metric (eqs. 2, 8)
    const float ir = frcp(r);
    const float ir3 = ir * ir * ir;
    const float x1R = sn * (r + 3.f * alpha * x2) * ir3;
    const float x1Z = (x2 * r + alpha * (3.f * x2 * x2 - 1.f)) * ir3;
    const float x2R = -x2 * sn * ir;
    const float x2Z = sn * sn * ir;
    const float ER = -(x1R * p1 + x2R * p2);
    const float EZ = -(x1Z * p1 + x2Z * p2);

    // Boris kick (eq. 9: dV_R = -omega V_Theta dt, dV_Theta = +omega V_R dt).
    // The rotation is applied as v + ((cos - 1) v + sin v_perp) with cos - 1
    // held separately, so its FP32 form preserves |v| to ~1e-10 per step
    // instead of drifting by the rounding of cos.
    vR += qmh * ER;
    vZ += qmh * EZ;
    {
        const float t = vR + (K.rcm1 * vR - K.rs * vT);
        vT = vT + (K.rs * vR + K.rcm1 * vT);
        vR = t;
    }
    vR += qmh * ER;
    vZ += qmh * EZ;

    // drift in the local Cartesian frame
    const float dX = step * vR, dY = step * vT, dZ = step * vZ;
    const float X = R + dX, Zn = Z + dZ;
    const float Rn2 = X * X + dY * dY;
    // rotation of (v_R, v_Theta) into the new meridional plane, again as
    // v + ((cos - 1) v + sin v_perp) with cos - 1 = -dY^2 / (R' (X + R'));
    // 1/R' and R' come from one reciprocal square root
    float cm = 0.f, sr = 0.f;
    if (Rn2 > 0.f) {
        const float iR = frsq(Rn2);
        const float Rn = Rn2 * iR;
        sr = dY * iR;
        cm = X > 0.f ? -(dY * dY) * iR * frcp(X + Rn) : X * iR - 1.f;
    }
    const float vRn = vR + (cm * vR + sr * vT);
    const float vTn = vT + (-sr * vR + cm * vT);

    // new conforming position from the displacement
    const float dr2 = 2.f * (R * dX + Z * dZ) + (dX * dX + dY * dY + dZ * dZ);  // r'^2 - r^2
    const float rn2 = Rn2 + Zn * Zn;
    const float irn = frsq(rn2);
    const float rn = rn2 * irn;
    const float dr = dr2 * frcp(rn + r);
    const float irr = ir * irn;
    const float dx2 = (dZ * r - Z * dr) * irr;
    const float dx1 = dr * irr - alpha * (dx2 * r * r - x2 * dr * (2.f * r + dr)) * irr * irr;
    const float t1 = f1 + dx1 * K.ih1;
    const float k1 = floorf(t1);
    i1n = i1 + (int)k1;
    f1n = t1 - k1;
    if (f1n >= 1.f) { f1n = 0.f; ++i1n; }
    const float t2 = f2 + dx2 * K.ih2;
    const float k2 = floorf(t2);
    i2n = i2 + (int)k2;
    f2n = t2 - k2;
    if (f2n >= 1.f) { f2n = 0.f; ++i2n; }
    if (i2n <= 0 || i2n >= n2 - 1) {
        // next to the axis: distance to it from 1 -+ x2' = R'^2 / (r' (r' +- Z'))
        if (Zn > 0.f) {
            const float u = Rn2 * frcp(rn * (rn + Zn)) * K.ih2;     // (1 - x2') / h2
            const float j = floorf(u);
            i2n = n2 - 1 - (int)j;
            f2n = 1.f - (u - j);
            if (f2n >= 1.f) { f2n = 0.f; ++i2n; }
        } else {
            const float u = Rn2 * frcp(rn * (rn - Zn)) * K.ih2;     // (1 + x2') / h2
            const float j = floorf(u);
            i2n = (int)j;
            f2n = u - j;
        }
        if (i2n < 0) { i2n = 0; f2n = 0.f; }
        if (i2n > n2 - 1) { i2n = n2 - 1; f2n = 0.99999994f; }
    }

    // boundaries: absorbed if the chord meets the grain (or, by rounding next
    // to the surface, only the end point lies inside: tallied there)
    const float t_hit = grain_chord<float>((float)gp.r_grain_max, alpha, R, Z, dX, dY, dZ, 24);
    const bool absorbed = i1n < 0 || t_hit >= 0.f;
    if (absorbed)
        tally_impact<float>(gp.n_bins, ImpactSpecies{sp.q, sp.m, sp.w, sp.e_bind}, s, ns, R, Z, dX,
                            dY, dZ, t_hit >= 0.f ? t_hit : 1.f, vR, vZ, vT, tally, tally_count);
    const int res = absorbed ? 1 : (i1n >= n1 ? 2 : 0);
    // every slot is written, a removed particle with the dead mark (its other
    // words are not read again): the stores need no branch
    st_stream(cell, res == 0 ? pack_cell(i1n, i2n) : DEAD);
    st_stream(slot4(static_cast<float*>(b.pos1), p), f1n);
    st_stream(slot4(static_cast<float*>(b.pos2), p), f2n);
    st_stream(slot4(static_cast<float*>(b.vR), p), vRn);
    st_stream(slot4(static_cast<float*>(b.vZ), p), vZ);
    st_stream(slot4(static_cast<float*>(b.vT), p), vTn);
    return res;
}

// ----------------------------------------------------------------- FP64 plain push
__device__ inline void locate64(const GrainParams& gp, double x1, double x2, int& i1, int& i2,
                                double& f1, double& f2) {
    const double t1 = (x1 + 1.0) * gp.inv_h1;
    const double t2 = (x2 + 1.0) * gp.inv_h2;
    i1 = (int)floor(t1);
    i2 = (int)floor(t2);
    i1 = i1 < 0 ? 0 : (i1 > gp.n1 - 1 ? gp.n1 - 1 : i1);
    i2 = i2 < 0 ? 0 : (i2 > gp.n2 - 1 ? gp.n2 - 1 : i2);
    f1 = t1 - i1;
    f2 = t2 - i2;
}

__device__ inline void deposit64(const GrainParams& gp, double* dep, double x1, double x2) {
    int i1, i2;
    double f1, f2;
    locate64(gp, x1, x2, i1, i2, f1, f2);
    const int o = i2 * gp.nx + i1;
    gadd(&dep[o], (1 - f1) * (1 - f2));
    gadd(&dep[o + 1], f1 * (1 - f2));
    gadd(&dep[o + gp.nx], (1 - f1) * f2);
    gadd(&dep[o + gp.nx + 1], f1 * f2);
}

// Drift, boundary test, tally: shared by the FP64 push and by injection.
// Returns 0 = alive (x1n/x2n/v written), 1 = absorbed, 2 = escaped.
__device__ inline int drift_and_bound64(const GrainParams& gp, const SpeciesParams& sp, int s,
                                        int ns, double R, double Z, double vR, double vZ,
                                        double vT, double step, double& x1n, double& x2n,
                                        double& vRn, double& vTn, double* tally,
                                        unsigned long long* tally_count) {
    const double dX = step * vR, dY = step * vT, dZ = step * vZ;
    const double X = R + dX, Zn = Z + dZ;
    const double Rn = sqrt(X * X + dY * dY);
    double cr = 1.0, sr = 0.0;
    if (Rn > 0.0) { cr = X / Rn; sr = dY / Rn; }
    vRn = cr * vR + sr * vT;
    vTn = -sr * vR + cr * vT;
    const double rn = sqrt(Rn * Rn + Zn * Zn);
    x2n = Zn / rn;
    x1n = x1_of(rn, x2n, gp.alpha);
    const double t_hit = grain_chord<double>(gp.r_grain_max, gp.alpha, R, Z, dX, dY, dZ, 60);
    if (!(x1n > -1.0) || t_hit >= 0.0) {
        tally_impact<double>(gp.n_bins, ImpactSpecies{sp.q, sp.m, sp.w, sp.e_bind}, s, ns, R, Z, dX,
                             dY, dZ, t_hit >= 0.0 ? t_hit : 1.0, vR, vZ, vT, tally, tally_count);
        return 1;
    }
    if (x1n >= gp.x1_out) return 2;
    return 0;
}

// One particle of the FP64 plain form; same return convention as the split form.
struct PlainState {
    double x1, x2, vR, vZ, vT;
};

__device__ inline PlainState load_plain(const PBuf& b, int64_t p) {
    PlainState q;
    q.x1 = gbl(static_cast<const double*>(b.pos1))[p];
    q.x2 = gbl(static_cast<const double*>(b.pos2))[p];
    q.vR = gbl(static_cast<const double*>(b.vR))[p];
    q.vZ = gbl(static_cast<const double*>(b.vZ))[p];
    q.vT = gbl(static_cast<const double*>(b.vT))[p];
    return q;
}

__device__ inline void set_dead(PlainState& q) { q.x1 = FP64_DEAD; }
__device__ inline bool is_dead(const PlainState& q) { return q.x1 > 0.0; }

__device__ inline int push_plain_one(const GrainParams& gp, const SpeciesParams& sp, int s, int ns,
                                     int64_t p, const PlainState& q, const PBuf& b,
                                     const double2* __restrict__ grad, double* __restrict__ tally,
                                     unsigned long long* __restrict__ tally_count, int& i1n,
                                     int& i2n, double& f1n, double& f2n) {
    const double x1 = q.x1;
    if (x1 > 0.0) return -1;
    const gptr<double> x1a = gbl(static_cast<double*>(b.pos1));
    const gptr<double> x2a = gbl(static_cast<double*>(b.pos2));
    const gptr<double> vRa = gbl(static_cast<double*>(b.vR));
    const gptr<double> vZa = gbl(static_cast<double*>(b.vZ));
    const gptr<double> vTa = gbl(static_cast<double*>(b.vT));
    const int nx = gp.nx;
    const double alpha = gp.alpha;
    const double x2 = q.x2;
    double vR = q.vR, vZ = q.vZ, vT = q.vT;
    int i1, i2;
    double f1, f2;
    locate64(gp, x1, x2, i1, i2, f1, f2);
    const int idx = i2 * nx + i1;
    const gptr<const double> gr = gbl(reinterpret_cast<const double*>(grad));
    const double2 g00 = make_double2(gr[2 * idx], gr[2 * idx + 1]);
    const double2 g10 = make_double2(gr[2 * idx + 2], gr[2 * idx + 3]);
    const double2 g01 = make_double2(gr[2 * (idx + nx)], gr[2 * (idx + nx) + 1]);
    const double2 g11 = make_double2(gr[2 * (idx + nx) + 2], gr[2 * (idx + nx) + 3]);
    const double w00 = (1 - f1) * (1 - f2), w10 = f1 * (1 - f2);
    const double w01 = (1 - f1) * f2, w11 = f1 * f2;
    const double p1 = w00 * g00.x + w10 * g10.x + w01 * g01.x + w11 * g11.x;
    const double p2 = w00 * g00.y + w10 * g10.y + w01 * g01.y + w11 * g11.y;
    const double r = r_of(x1, x2, alpha);
    const double sn = sqrt(fmax(1.0 - x2 * x2, 0.0));
    const double R = r * sn, Z = r * x2;
    const Metric<double> m = metric_at(r, x2, sn, alpha);
    const double ER = -(m.x1R * p1 + m.x2R * p2);
    const double EZ = -(m.x1Z * p1 + m.x2Z * p2);
    vR += sp.qm_half * ER;
    vZ += sp.qm_half * EZ;
    {
        const double t = sp.rot_c * vR - sp.rot_s * vT;
        vT = sp.rot_s * vR + sp.rot_c * vT;
        vR = t;
    }
    vR += sp.qm_half * ER;
    vZ += sp.qm_half * EZ;
    double x1n, x2n, vRn, vTn;
    const int st = drift_and_bound64(gp, sp, s, ns, R, Z, vR, vZ, vT, gp.step, x1n, x2n, vRn, vTn,
                                     tally, tally_count);
    if (st != 0) {
        x1a[p] = FP64_DEAD;
        return st;
    }
    st_stream(x1a + p, x1n);
    st_stream(x2a + p, x2n);
    st_stream(vRa + p, vRn);
    st_stream(vZa + p, vZ);
    st_stream(vTa + p, vTn);
    locate64(gp, x1n, x2n, i1n, i2n, f1n, f2n);
    return 0;
}

// ----------------------------------------------------------------- ensemble push
// One persistent launch pushes every (grain, species) task of the context.  The
// tasks' particle slots are cut into chunks of PB * NT consecutive
// (tile-sorted) particles; k_plan_chunks lays the chunks of all tasks end to
// end.  The chunk range is split into eight contiguous parts, one per XCD
// (workgroup b runs on XCD b mod 8), so that the chunks of neighbouring tiles,
// which read the same field nodes and add into the same deposit nodes, share
// one L2.  A workgroup loads the packed cells of its chunk first, derives the
// chunk's deposit window from them, then advances the particles (each one's
// state loading while the one before it is advanced) and deposits their
// charge into an LDS window of nodes; the window's non-zero nodes are added to
// the global deposit array once per chunk.
template <bool SPLIT> struct PushTraits;
template <> struct PushTraits<true> {
    using S = SplitState;
    using T = float;
    using A = unsigned long long;   // two 32-bit fixed-point sums per LDS word
    static constexpr int PB = 8;    // particles per thread and chunk (even)
    // eight waves, two workgroups per CU at four waves per SIMD: a chunk of
    // 4096 particles shares one deposit window, so a particle pays half the
    // window flushes and chunk-start barriers of a 256-thread workgroup
    static constexpr int NT = 512;
};
template <> struct PushTraits<false> {
    using S = PlainState;
    using T = double;
    using A = double;
    static constexpr int PB = 4;
    // 174 registers allow eight waves per CU whatever the workgroup size; two
    // 256-thread workgroups per CU overlap each other's serial phases
    static constexpr int NT = 256;
};

constexpr int WIN_CAP = 4096;
constexpr int WIN_MARGIN = 4;

int push_chunk(bool split) {
    return split ? PushTraits<true>::NT * PushTraits<true>::PB : PushTraits<false>::NT * PushTraits<false>::PB;
}

// chunks of every task, laid end to end: prefix[t] = first chunk of task t
__global__ void __launch_bounds__(BLOCK)
k_plan_chunks(const PushTask* __restrict__ tasks, int ntasks, int64_t chunk, int64_t* __restrict__ prefix) {
    __shared__ int64_t cnt[BLOCK];
    int64_t carry = 0;
    for (int t0 = 0; t0 < ntasks; t0 += BLOCK) {
        const int t = t0 + threadIdx.x;
        int64_t c = 0;
        if (t < ntasks) {
            const PushTask& T = tasks[t];
            c = (T.ctr->n[T.s] + chunk - 1) / chunk;
        }
        cnt[threadIdx.x] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int k = 0; k < BLOCK && t0 + k < ntasks; ++k) {
                prefix[t0 + k] = carry;
                carry += cnt[k];
            }
            prefix[min(t0 + BLOCK, ntasks)] = carry;
        }
        __syncthreads();
        carry = prefix[min(t0 + BLOCK, ntasks)];
        __syncthreads();
    }
}

// task of chunk c: the largest t with prefix[t] <= c
__device__ inline int find_task(const int64_t* __restrict__ prefix, int ntasks, int64_t c) {
    int lo = 0, hi = ntasks;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= c) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Bounding box of a chunk's cells, held as two packed cell words (the key
// layout, i2 << 16 | i1): the componentwise 16-bit minimum and maximum.  The
// empty box is lo = all ones, hi = 0; a dead key (all ones) leaves the minimum
// as it is and is masked out of the maximum.
using u16x2 = unsigned short __attribute__((ext_vector_type(2)));
__device__ inline uint32_t pk_min16(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}
__device__ inline uint32_t pk_max16(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}

struct Box {
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
};
__device__ inline void box_add(Box& b, int32_t c) {
    b.lo = pk_min16(b.lo, (uint32_t)c);
    b.hi = pk_max16(b.hi, c < 0 ? 0u : (uint32_t)c);
}

// Over the wave: within each row of 16 lanes by DPP (the quad swaps [1,0,3,2]
// and [2,3,0,1], then row rotations by 4 and 8 lanes), across the four rows by
// two xor shuffles.  Called with every lane active.
template <bool MAX>
__device__ inline uint32_t wave_box(uint32_t x) {
    auto op = [](uint32_t a, uint32_t b) { return MAX ? pk_max16(a, b) : pk_min16(a, b); };
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0xB1, 0xF, 0xF, false));
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x4E, 0xF, 0xF, false));
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x124, 0xF, 0xF, false));
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x128, 0xF, 0xF, false));
    x = op(x, (uint32_t)__shfl_xor((int)x, 16));
    x = op(x, (uint32_t)__shfl_xor((int)x, 32));
    return x;
}

template <int NT>
__device__ inline Box block_box(Box b, uint32_t (*red)[NT / 64]) {
    b.lo = wave_box<false>(b.lo);
    b.hi = wave_box<true>(b.hi);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = b.lo;
        red[1][w] = b.hi;
    }
    __syncthreads();
    b.lo = red[0][0];
    b.hi = red[1][0];
    for (int q = 1; q < NT / 64; ++q) {
        b.lo = pk_min16(b.lo, red[0][q]);
        b.hi = pk_max16(b.hi, red[1][q]);
    }
    __syncthreads();
    return b;
}

// Deposit window of one chunk: the bounding box of the chunk's current cells
// widened by WIN_MARGIN cells on every side (clipped to the grid), or, if that
// exceeds the LDS capacity, a 64-column window around the box's centre.
// Particles whose new cell falls outside go straight to global atomics.
struct Window {
    int wi0, wj0, W, H, C;   // first node, extent in nodes, lane-striped copies
    bool on;
};

__device__ inline bool state_cell(const GrainParams&, const SplitState& q, int& i1, int& i2) {
    if (q.c < 0) return false;
    i1 = cell_i1(q.c);
    i2 = cell_i2(q.c);
    return true;
}

__device__ inline bool state_cell(const GrainParams& gp, const PlainState& q, int& i1, int& i2) {
    if (q.x1 > 0.0) return false;
    double f1, f2;
    locate64(gp, q.x1, q.x2, i1, i2, f1, f2);
    return true;
}

// Window from the chunk's bounding box (each lane's part in b).
template <int NT>
__device__ inline Window window_from(const GrainParams& gp, Box b, uint32_t (*red)[NT / 64]) {
    b = block_box<NT>(b, red);
    const int i1a = cell_i1((int32_t)b.lo), i1b = cell_i1((int32_t)b.hi);
    const int i2a = cell_i2((int32_t)b.lo), i2b = cell_i2((int32_t)b.hi);
    Window w;
    w.on = i1a <= i1b;
    if (!w.on) return w;
    const int nx = gp.nx, ny = gp.n2 + 1;
    w.wi0 = max(i1a - WIN_MARGIN, 0);
    w.wj0 = max(i2a - WIN_MARGIN, 0);
    w.W = min(i1b + WIN_MARGIN + 1, gp.n1) - w.wi0 + 1;
    w.H = min(i2b + WIN_MARGIN + 1, gp.n2) - w.wj0 + 1;
    if (w.W * w.H > WIN_CAP) {
        w.W = min(w.W, 64);
        w.H = min(w.H, WIN_CAP / w.W);
        w.wi0 = max(0, min((i1a + i1b) / 2 - w.W / 2, nx - w.W));
        w.wj0 = max(0, min((i2a + i2b) / 2 - w.H / 2, ny - w.H));
    }
    // Up to 16 lane-striped copies of every window node (copy = lane mod C; the
    // copies of a node sit in consecutive LDS banks): particles of one wave
    // landing on the same node add into different words instead of
    // serialising on one address.
    w.C = 16;
    while (w.C > 1 && w.W * w.H * w.C > WIN_CAP) w.C >>= 1;
    return w;
}

template <int NT, typename S, int PB>
__device__ inline Window chunk_window(const GrainParams& gp, const S (&st)[PB], uint32_t (*red)[NT / 64]) {
    Box b;
#pragma unroll
    for (int k = 0; k < PB; ++k) {
        int i1, i2;
        if (state_cell(gp, st[k], i1, i2)) box_add(b, pack_cell(i1, i2));
    }
    return window_from<NT>(gp, b, red);
}

// FP64 form: one double per node copy.
__device__ inline void deposit_one(const GrainParams& gp, const Window& w, double* __restrict__ win,
                                   double* __restrict__ dep, int i1, int i2, double f1, double f2) {
    const double a1 = 1.0 - f1, a2 = 1.0 - f2;
    const double w00 = a1 * a2, w10 = f1 * a2, w01 = a1 * f2, w11 = f1 * f2;
    const int li = i1 - w.wi0, lj = i2 - w.wj0;
    if (li >= 0 && li < w.W - 1 && lj >= 0 && lj < w.H - 1) {
        const int C = w.C, cp = threadIdx.x & (C - 1);
        const int o = lj * w.W + li;
        atomicAdd(&win[o * C + cp], w00);
        atomicAdd(&win[(o + 1) * C + cp], w10);
        atomicAdd(&win[(o + w.W) * C + cp], w01);
        atomicAdd(&win[(o + w.W + 1) * C + cp], w11);
    } else {
        const int nx = gp.nx;
        const int o = i2 * nx + i1;
        gadd(&dep[o], w00);
        gadd(&dep[o + 1], w10);
        gadd(&dep[o + nx], w01);
        gadd(&dep[o + nx + 1], w11);
    }
}

__device__ inline void flush_window(const GrainParams& gp, const Window& w, double* __restrict__ win,
                                    double* __restrict__ dep) {
    const int nodes_w = w.W * w.H, C = w.C, nx = gp.nx;
    for (int q = threadIdx.x; q < nodes_w; q += PushTraits<false>::NT) {
        double val = 0.0;
        for (int c = 0; c < C; ++c) {
            const int a = q * C + ((c + q) & (C - 1));
            val += win[a];
            win[a] = 0.0;
        }
        if (val != 0.0) {
            const int row = q / w.W;
            gadd(&dep[(w.wj0 + row) * nx + w.wi0 + (q - row * w.W)], val);
        }
    }
}

// FP32 split form: the window holds 64-bit words of two 32-bit fixed-point
// sums, the left and the right node of a cell edge (word o = nodes o, o + 1).
// A particle then needs two integer LDS atomics (bottom and top edge of its
// cell) instead of four float ones, and the window sums do not depend on the
// order of the additions.  With C copies a copy receives at most CHUNK / C
// particles, each adding at most 1: the fraction bits 31 - log2(CHUNK / C)
// keep every 32-bit sum below 2^31 (2^-19 .. 2^-23 for CHUNK = 4096).
constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }
constexpr int SPLIT_CHUNK_LOG2 = ilog2(PushTraits<true>::PB * PushTraits<true>::NT);
__device__ inline int fx_bits(int C) { return 31 - SPLIT_CHUNK_LOG2 + (31 - __clz(C)); }

__device__ inline void deposit_one(const GrainParams& gp, const Window& w,
                                   unsigned long long* __restrict__ win, float* __restrict__ dep,
                                   int i1, int i2, float f1, float f2) {
    const float a1 = 1.f - f1, a2 = 1.f - f2;
    const float w00 = a1 * a2, w10 = f1 * a2, w01 = a1 * f2, w11 = f1 * f2;
    const int li = i1 - w.wi0, lj = i2 - w.wj0;
    if (li >= 0 && li < w.W - 1 && lj >= 0 && lj < w.H - 1) {
        const int C = w.C, cp = threadIdx.x & (C - 1);
        const float sc = (float)(1 << fx_bits(C));
        const unsigned long long bot =
            (unsigned long long)(uint32_t)(w00 * sc + 0.5f) | ((unsigned long long)(uint32_t)(w10 * sc + 0.5f) << 32);
        const unsigned long long top =
            (unsigned long long)(uint32_t)(w01 * sc + 0.5f) | ((unsigned long long)(uint32_t)(w11 * sc + 0.5f) << 32);
        const int o = lj * w.W + li;
        atomicAdd(&win[o * C + cp], bot);
        atomicAdd(&win[(o + w.W) * C + cp], top);
    } else {
        const int nx = gp.nx;
        const int o = i2 * nx + i1;
        gadd(&dep[o], w00);
        gadd(&dep[o + 1], w10);
        gadd(&dep[o + nx], w01);
        gadd(&dep[o + nx + 1], w11);
    }
}

__device__ inline void flush_window(const GrainParams& gp, const Window& w,
                                    unsigned long long* __restrict__ win, float* __restrict__ dep) {
    const int nodes_w = w.W * w.H, C = w.C, nx = gp.nx;
    const double isc = 1.0 / (double)(1 << fx_bits(C));
    for (int q = threadIdx.x; q < nodes_w; q += PushTraits<true>::NT) {
        const int row = q / w.W, col = q - row * w.W;
        unsigned long long sum = 0;
        for (int c = 0; c < C; ++c) sum += win[q * C + ((c + q) & (C - 1))] & 0xFFFFFFFFull;
        if (col > 0)
            for (int c = 0; c < C; ++c) sum += win[(q - 1) * C + ((c + q) & (C - 1))] >> 32;
        if (sum) gadd(&dep[(w.wj0 + row) * nx + w.wi0 + col], (float)((double)sum * isc));
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nodes_w * C; q += PushTraits<true>::NT) win[q] = 0ull;
}

__device__ inline SplitState load_state(const PBuf& b, int64_t p, SplitState*) { return load_split(b, p); }
__device__ inline PlainState load_state(const PBuf& b, int64_t p, PlainState*) { return load_plain(b, p); }

// chunk range of this workgroup's XCD: [lo, hi), stride = workgroups per XCD
__device__ inline void xcd_range(int64_t total, int64_t& first, int64_t& hi, int& stride) {
    const int xcd = blockIdx.x & 7;
    stride = gridDim.x >> 3;
    const int64_t lo = total * xcd / 8;
    hi = total * (xcd + 1) / 8;
    first = lo + (blockIdx.x >> 3);
}

// Parameters of the task a workgroup is working on, reloaded only when its
// chunk index crosses into the next task (the chunk index only grows), so the
// chain prefix -> task -> counters -> buffers is paid once per task, not per
// chunk.
template <typename T>
struct TaskView {
    GrainParams gp;
    SpeciesParams sp;
    PBuf b;
    const void* grad;
    T* dep;
    DevCounters* ctr;
    double* tally;
    unsigned long long* tally_count;
    int64_t n, first_chunk, end_chunk;
    int s, ns;
};

template <typename T>
__device__ inline void load_task(const PushTask* __restrict__ tasks, const int64_t* __restrict__ prefix,
                                 int ntasks, int64_t c, bool deposit, TaskView<T>& v) {
    const int t = find_task(prefix, ntasks, c);
    const PushTask& task = tasks[t];
    v.first_chunk = prefix[t];
    v.end_chunk = prefix[t + 1];
    v.gp = task.gp;
    v.sp = task.sp;
    v.ctr = task.ctr;
    v.s = task.s;
    v.ns = task.ns;
    v.grad = task.grad;
    v.dep = deposit ? static_cast<T*>(task.dep) : nullptr;
    v.tally = task.tally;
    v.tally_count = task.tally_count;
    // the live count and buffer index come from memory this kernel also
    // writes (vector loads); they are the same in every lane, and reading them
    // into scalar registers keeps the task's array bases scalar as well
    const int64_t n = v.ctr->n[v.s];
    v.n = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(n >> 32)) << 32) |
                    (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)n));
    v.b = task.buf[__builtin_amdgcn_readfirstlane(v.ctr->cur[v.s])];
}

__device__ inline void flush_counts(DevCounters* ctr, int s, uint32_t& n_live, uint32_t& n_abs, uint32_t& n_esc) {
    block_count_add(n_live, reinterpret_cast<unsigned long long*>(&ctr->pushed[s]));
    block_count_add(n_abs, reinterpret_cast<unsigned long long*>(&ctr->absorbed[s]));
    block_count_add(n_esc, reinterpret_cast<unsigned long long*>(&ctr->escaped[s]));
    n_live = n_abs = n_esc = 0;
}

// Loading a chunk: the keys (packed cell / FP64 position) of all its particles
// first -- the deposit window needs them before anything else -- then the rest
// of each particle's state (and, FP32, its cell's nodal gradients) one
// particle ahead inside a rolled loop of two particles per iteration, which
// keeps the loads in flight per wave close to what the HBM pipe needs without
// inflating the register count.

struct SplitKey { int32_t c; };
struct PlainKey { double x1, x2; };

__device__ inline void load_key(const PBuf& b, int64_t p, int64_t n, SplitKey& k) {
    k.c = p < n ? ld_stream(slot4(static_cast<const int32_t*>(b.pos0), p)) : DEAD;
}
__device__ inline void load_key(const PBuf& b, int64_t p, int64_t n, PlainKey& k) {
    if (p < n) {
        k.x1 = ld_stream(gbl(static_cast<const double*>(b.pos1)) + p);
        k.x2 = ld_stream(gbl(static_cast<const double*>(b.pos2)) + p);
    } else {
        k.x1 = FP64_DEAD;
        k.x2 = 0.0;
    }
}

__device__ inline bool key_cell(const GrainParams&, const SplitKey& k, int& i1, int& i2) {
    if (k.c < 0) return false;
    i1 = cell_i1(k.c);
    i2 = cell_i2(k.c);
    return true;
}
__device__ inline bool key_cell(const GrainParams& gp, const PlainKey& k, int& i1, int& i2) {
    if (k.x1 > 0.0) return false;
    double f1, f2;
    locate64(gp, k.x1, k.x2, i1, i2, f1, f2);
    return true;
}

// the state besides the key; loaded whenever the slot exists, so the loads
// need not wait for the key
__device__ inline void load_fields(const PBuf& b, int64_t p, int64_t n, SplitState& q) {
    if (p >= n) return;
    q.f1 = ld_stream(slot4(static_cast<const float*>(b.pos1), p));
    q.f2 = ld_stream(slot4(static_cast<const float*>(b.pos2), p));
    q.vR = ld_stream(slot4(static_cast<const float*>(b.vR), p));
    q.vZ = ld_stream(slot4(static_cast<const float*>(b.vZ), p));
    q.vT = ld_stream(slot4(static_cast<const float*>(b.vT), p));
}
__device__ inline void load_fields(const PBuf& b, int64_t p, int64_t n, PlainState& q) {
    if (p >= n) return;
    q.vR = ld_stream(gbl(static_cast<const double*>(b.vR)) + p);
    q.vZ = ld_stream(gbl(static_cast<const double*>(b.vZ)) + p);
    q.vT = ld_stream(gbl(static_cast<const double*>(b.vT)) + p);
}

__device__ inline void set_key(SplitState& q, const SplitKey& k) { q.c = k.c; }

// The four float2 nodal gradients around the particle's cell, read as 64-bit
// words (the vector type cannot be copied out of an explicitly global
// reference); issued together with the state loads, one particle ahead, so the
// gather's latency overlaps the previous particle's work.
__device__ inline void load_gather(const void* grad, int nx, const SplitKey& k, SplitState& q) {
    if (k.c < 0) return;
    const int idx = cell_i2(k.c) * nx + cell_i1(k.c);
    const gptr<const unsigned long long> gr = gbl(static_cast<const unsigned long long*>(grad));
    q.g[0] = gr[idx];
    q.g[1] = gr[idx + 1];
    q.g[2] = gr[idx + nx];
    q.g[3] = gr[idx + nx + 1];
}
__device__ inline void load_gather(const void*, int, const PlainKey&, PlainState&) {}
__device__ inline void set_key(PlainState& q, const PlainKey& k) {
    q.x1 = k.x1;
    q.x2 = k.x2;
}

// a split key is the packed cell itself (dead: all ones)
__device__ inline void box_key(const GrainParams&, const SplitKey& k, Box& b) { box_add(b, k.c); }
__device__ inline void box_key(const GrainParams& gp, const PlainKey& k, Box& b) {
    int i1, i2;
    if (key_cell(gp, k, i1, i2)) box_add(b, pack_cell(i1, i2));
}

template <int NT, typename K, int PB>
__device__ inline Window keys_window(const GrainParams& gp, const K (&key)[PB], uint32_t (*red)[NT / 64]) {
    Box b;
#pragma unroll
    for (int k = 0; k < PB; ++k) box_key(gp, key[k], b);
    return window_from<NT>(gp, b, red);
}

template <bool SPLIT> struct KeyOf;
template <> struct KeyOf<true> { using K = SplitKey; };
template <> struct KeyOf<false> { using K = PlainKey; };

template <bool SPLIT>
__device__ __forceinline__ void push_chunks(const PushTask* __restrict__ tasks, const int64_t* __restrict__ prefix,
                                            int ntasks, int deposit) {
    using Tr = PushTraits<SPLIT>;
    using S = typename Tr::S;
    using T = typename Tr::T;
    using A = typename Tr::A;
    using Key = typename KeyOf<SPLIT>::K;
    constexpr int PB = Tr::PB;
    constexpr int NT = Tr::NT;
    constexpr int CHUNK = PB * NT;
    __shared__ A win[WIN_CAP];
    __shared__ uint32_t red[2][NT / 64];
    for (int q = threadIdx.x; q < WIN_CAP; q += NT) win[q] = A(0);
    __syncthreads();
    int64_t c, hi;
    int stride;
    xcd_range(prefix[ntasks], c, hi, stride);
    TaskView<T> v;
    v.end_chunk = -1;
    v.ctr = nullptr;
    SplitConsts K;
    uint32_t n_live = 0, n_abs = 0, n_esc = 0;
    for (; c < hi; c += stride) {
        if (c >= v.end_chunk) {
            if (v.ctr) flush_counts(v.ctr, v.s, n_live, n_abs, n_esc);
            load_task(tasks, prefix, ntasks, c, deposit != 0, v);
            if constexpr (SPLIT) K = split_consts(v.gp, v.sp);
        }
        const int64_t base = (c - v.first_chunk) * CHUNK + threadIdx.x;
        Key key[PB];
#pragma unroll
        for (int k = 0; k < PB; ++k) load_key(v.b, base + k * NT, v.n, key[k]);
        // the first particle's state loads while the window is reduced
        S buf[2];
        load_fields(v.b, base, v.n, buf[0]);
        load_gather(v.grad, v.gp.nx, key[0], buf[0]);
        Window w;
        w.on = false;
        if (v.dep) w = keys_window<NT>(v.gp, key, red);
        auto advance = [&](int64_t p, S cur, const Key& kk) {
            set_key(cur, kk);
            int ia, ic;
            T f, g;
            int r;
            if constexpr (SPLIT)
                r = push_split_one(v.gp, v.sp, K, v.s, v.ns, p, cur, v.b, v.tally, v.tally_count, ia, ic, f, g);
            else
                r = push_plain_one(v.gp, v.sp, v.s, v.ns, p, cur, v.b,
                                   static_cast<const double2*>(v.grad), v.tally, v.tally_count, ia, ic, f, g);
            if (r < 0) return;
            ++n_live;
            if (r == 1) { ++n_abs; return; }
            if (r == 2) { ++n_esc; return; }
            if (w.on) deposit_one(v.gp, w, win, v.dep, ia, ic, f, g);
        };
        // two particles per iteration with two state buffers: each particle's
        // state and gather load while the one before it is advanced, and no
        // buffer is copied (a copy would wait for the loads it moves)
#pragma unroll 1
        for (int k = 0; k < PB; k += 2) {
            const int64_t p = base + k * NT;
            load_fields(v.b, p + NT, v.n, buf[1]);
            load_gather(v.grad, v.gp.nx, key[1], buf[1]);
            advance(p, buf[0], key[0]);
            if (k + 2 < PB) {
                load_fields(v.b, p + 2 * NT, v.n, buf[0]);
                load_gather(v.grad, v.gp.nx, key[2], buf[0]);
            }
            advance(p + NT, buf[1], key[1]);
#pragma unroll
            for (int a = 0; a + 2 < PB; ++a) key[a] = key[a + 2];
        }
        if (w.on) {
            // the next chunk's window reduction synchronises before anything
            // is deposited again, which also covers the clearing of this window
            __syncthreads();
            flush_window(v.gp, w, win, v.dep);
        }
    }
    if (v.ctr) flush_counts(v.ctr, v.s, n_live, n_abs, n_esc);
}

// FP32: capped at 128 registers so four waves per SIMD stay resident (the
// kernel is bound by memory latency); FP64 keeps its registers.
__global__ void __launch_bounds__(PushTraits<true>::NT) __attribute__((amdgpu_waves_per_eu(4)))
k_push_split(const PushTask* __restrict__ tasks, const int64_t* __restrict__ prefix, int ntasks, int deposit) {
    push_chunks<true>(tasks, prefix, ntasks, deposit);
}

__global__ void __launch_bounds__(PushTraits<false>::NT)
k_push_plain(const PushTask* __restrict__ tasks, const int64_t* __restrict__ prefix, int ntasks, int deposit) {
    push_chunks<false>(tasks, prefix, ntasks, deposit);
}

// ----------------------------------------------------------------- deposit only
// Deposit of the current particles of every task (initial field, standalone
// solves) with the same chunks and windows as the push.
__device__ inline void state_offsets(const GrainParams&, const SplitState& q, int& i1, int& i2, float& f1, float& f2) {
    i1 = cell_i1(q.c);
    i2 = cell_i2(q.c);
    f1 = q.f1;
    f2 = q.f2;
}

__device__ inline void state_offsets(const GrainParams& gp, const PlainState& q, int& i1, int& i2, double& f1,
                                     double& f2) {
    locate64(gp, q.x1, q.x2, i1, i2, f1, f2);
}

template <bool SPLIT>
__global__ void __launch_bounds__(PushTraits<SPLIT>::NT)
k_deposit(const PushTask* __restrict__ tasks, const int64_t* __restrict__ prefix, int ntasks) {
    using Tr = PushTraits<SPLIT>;
    using S = typename Tr::S;
    using T = typename Tr::T;
    using A = typename Tr::A;
    constexpr int PB = Tr::PB;
    constexpr int NT = Tr::NT;
    constexpr int CHUNK = PB * NT;
    __shared__ A win[WIN_CAP];
    __shared__ uint32_t red[2][NT / 64];
    for (int q = threadIdx.x; q < WIN_CAP; q += NT) win[q] = A(0);
    __syncthreads();
    int64_t c, hi;
    int stride;
    xcd_range(prefix[ntasks], c, hi, stride);
    for (; c < hi; c += stride) {
        const int t = find_task(prefix, ntasks, c);
        const PushTask& task = tasks[t];
        const GrainParams gp = task.gp;
        const int s = task.s;
        const int64_t n = task.ctr->n[s];
        const PBuf b = task.buf[task.ctr->cur[s]];
        T* dep = static_cast<T*>(task.dep);
        const int64_t base = (c - prefix[t]) * CHUNK;
        S st[PB];
#pragma unroll
        for (int k = 0; k < PB; ++k) {
            const int64_t p = base + k * NT + threadIdx.x;
            if (p < n) st[k] = load_state(b, p, (S*)nullptr);
            else set_dead(st[k]);
        }
        const Window w = chunk_window<NT>(gp, st, red);
        if (!w.on) continue;
#pragma unroll
        for (int k = 0; k < PB; ++k) {
            if (is_dead(st[k])) continue;
            int i1, i2;
            T f1, f2;
            state_offsets(gp, st[k], i1, i2, f1, f2);
            deposit_one(gp, w, win, dep, i1, i2, f1, f2);
        }
        __syncthreads();
        flush_window(gp, w, win, dep);
        __syncthreads();
    }
}

// ----------------------------------------------------------------- store helpers
// Writes one particle given in FP64 conforming coordinates into either form.
__device__ inline void store_particle(const GrainParams& gp, bool split, const PBuf& b, int64_t p,
                                      double x1, double x2, double vR, double vZ, double vT) {
    if (split) {
        int i1, i2;
        double f1, f2;
        locate64(gp, x1, x2, i1, i2, f1, f2);
        float ff1 = (float)f1, ff2 = (float)f2;
        if (ff1 >= 1.f) ff1 = 0.99999994f;
        if (ff2 >= 1.f) ff2 = 0.99999994f;
        gbl(static_cast<int32_t*>(b.pos0))[p] = pack_cell(i1, i2);
        gbl(static_cast<float*>(b.pos1))[p] = ff1;
        gbl(static_cast<float*>(b.pos2))[p] = ff2;
        gbl(static_cast<float*>(b.vR))[p] = (float)vR;
        gbl(static_cast<float*>(b.vZ))[p] = (float)vZ;
        gbl(static_cast<float*>(b.vT))[p] = (float)vT;
    } else {
        gbl(static_cast<double*>(b.pos1))[p] = x1;
        gbl(static_cast<double*>(b.pos2))[p] = x2;
        gbl(static_cast<double*>(b.vR))[p] = vR;
        gbl(static_cast<double*>(b.vZ))[p] = vZ;
        gbl(static_cast<double*>(b.vT))[p] = vT;
    }
}

__device__ inline void store_dead(bool split, const PBuf& b, int64_t p) {
    if (split) gbl(static_cast<int32_t*>(b.pos0))[p] = DEAD;
    else gbl(static_cast<double*>(b.pos1))[p] = FP64_DEAD;
}

// ----------------------------------------------------------------- volume load
// Positions uniform in physical volume: x2 by rejection on r_out^3 - r_in^3,
// then r^3 uniform in [r_in^3, r_out^3]; Maxwellian velocities (Box-Muller).
__global__ void __launch_bounds__(BLOCK)
k_load(GrainParams gp, SpeciesParams sp, int s, int64_t n, bool split, PBuf b) {
    const double alpha = gp.alpha, xo = gp.x1_out;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        double x2 = 0, r3 = 0;
        for (int a = 0; a < MAX_ATTEMPTS; ++a) {
            const U4 u = philox4x32_10(U4{LOAD_STREAM, (uint32_t)s | (P_LOAD_POS << 8), (uint32_t)k,
                                          (uint32_t)a}, gp.key0, gp.key1);
            const double cx2 = -1.0 + 2.0 * unit_open(u.x);
            const double ri = r_of(-1.0, cx2, alpha), ro = r_of(xo, cx2, alpha);
            const double rin3 = ri * ri * ri, rout3 = ro * ro * ro;
            if (unit_open(u.y) * gp.M_vol <= (rout3 - rin3) || a == MAX_ATTEMPTS - 1) {
                x2 = cx2;
                r3 = rin3 + unit_open(u.z) * (rout3 - rin3);
                break;
            }
        }
        const double r = cbrt(r3);
        const double x1 = x1_of(r, x2, alpha);
        const U4 v = philox4x32_10(U4{LOAD_STREAM, (uint32_t)s | (P_LOAD_VEL << 8), (uint32_t)k, 0u},
                                   gp.key0, gp.key1);
        const double g0 = sqrt(-2.0 * log(unit_open(v.x)));
        const double g1 = sqrt(-2.0 * log(unit_open(v.z)));
        const double tp = 6.283185307179586;
        const double vR = sp.sigma * g0 * cos(tp * unit_open(v.y));
        const double vZ = sp.sigma * g0 * sin(tp * unit_open(v.y));
        const double vT = sp.sigma * g1 * cos(tp * unit_open(v.w));
        store_particle(gp, split, b, k, x1, x2, vR, vZ, vT);
        gbl(b.id)[k] = (uint32_t)k;
    }
}

// Host-given particles (already copied to device FP64 arrays).
__global__ void __launch_bounds__(BLOCK)
k_set(GrainParams gp, int64_t n, bool split, PBuf b, const double* __restrict__ x1,
      const double* __restrict__ x2, const double* __restrict__ vR,
      const double* __restrict__ vZ, const double* __restrict__ vT, int* bad) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double a = x1[k], c = x2[k];
        if (!(a > -1.0 && a < gp.x1_out && c >= -1.0 && c <= 1.0)) {
            __hip_atomic_fetch_or(gbl(bad), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            store_dead(split, b, k);
        } else {
            store_particle(gp, split, b, k, a, c, vR[k], vZ[k], vT[k]);
        }
        gbl(b.id)[k] = (uint32_t)k;
    }
}

// ----------------------------------------------------------------- injection
// Per task: the step's count from the 2^-32 fixed-point accumulator (exact
// integers), the slots it takes (capacity permitting; the excess sets the
// sticky overflow flag), its first id and the Philox stream (= the grain's
// step index).
__global__ void __launch_bounds__(BLOCK)
k_inject_plan(const PushTask* __restrict__ tasks, int ntasks) {
    for (int t = threadIdx.x; t < ntasks; t += BLOCK) {
        const PushTask& T = tasks[t];
        DevCounters* ctr = T.ctr;
        const int s = T.s;
        const uint64_t acc = ctr->inj_acc[s] + T.inj_inc;
        const int64_t n_new = (int64_t)(acc >> 32);
        ctr->inj_acc[s] = acc & 0xFFFFFFFFull;
        const int64_t n = ctr->n[s];
        const int64_t room = T.capacity > n ? T.capacity - n : 0;
        const int64_t placed = n_new < room ? n_new : room;
        if (placed < n_new) ctr->overflow = 1u;
        ctr->inj_base[s] = n;
        ctr->inj_new[s] = n_new;
        ctr->inj_id0[s] = ctr->next_id[s];
        ctr->n[s] = n + placed;
        ctr->injected[s] += (uint64_t)placed;
        ctr->next_id[s] += (uint32_t)n_new;
        if (s == 0) {
            ctr->inj_tag = (uint32_t)(ctr->step & 0xFFFFFFFFull);
            ctr->step += 1;
        }
    }
}

// Flux-Maxwellian injection at x1_out: x2 with density proportional to eq. (4),
// inward normal speed Rayleigh(sigma), tangential normal(0, sigma^2), then a
// straight partial step U * dt with the usual boundary tests; the survivors
// deposit their charge.  Slot = base + k, id = id0 + k.  A workgroup takes
// INJ_PER_BLOCK consecutive particles of one task; the tasks' workgroups are
// laid end to end (block_task), each task with as many as its largest
// injection needs.  The injected particles end their partial step within a
// cell of the outer boundary, so every step's injections deposit onto the same
// three node columns: a workgroup adds its particles' weights in LDS and then
// each node once to the global sums, instead of thousands of workgroups'
// atomics contending on those few hundred nodes.
__global__ void __launch_bounds__(INJ_BLOCK)
k_inject(const PushTask* __restrict__ tasks, const int* __restrict__ block_task, bool split, int deposit) {
    extern __shared__ unsigned char inj_lds[];
    const PushTask& T = tasks[block_task[blockIdx.x]];
    const GrainParams gp = T.gp;
    const SpeciesParams sp = T.sp;
    DevCounters* ctr = T.ctr;
    const int s = T.s, ns = T.ns;
    const int64_t n_new = ctr->inj_new[s];
    const int64_t base = ctr->inj_base[s];
    const uint32_t id0 = ctr->inj_id0[s];
    const uint32_t stream_tag = ctr->inj_tag;
    const PBuf b = T.buf[ctr->cur[s]];
    void* dep = deposit ? T.dep : nullptr;
    double* tally = T.tally;
    unsigned long long* tally_count = T.tally_count;
    const double alpha = gp.alpha, xo = gp.x1_out;
    uint32_t n_abs = 0, n_esc = 0;
    // node window: columns n1 - 2 .. n1 of every row, [row][3]
    const int n1 = gp.n1, nx = gp.nx, wn = 3 * (gp.n2 + 1);
    float* wf = reinterpret_cast<float*>(inj_lds);
    double* wd = reinterpret_cast<double*>(inj_lds);
    if (dep) {
        for (int q = threadIdx.x; q < wn; q += INJ_BLOCK) {
            if (split) wf[q] = 0.f;
            else wd[q] = 0.0;
        }
        __syncthreads();
    }
    const int64_t k0 = (int64_t)(blockIdx.x - T.inj_block0) * INJ_PER_BLOCK;
    const int64_t k_end = k0 + INJ_PER_BLOCK < n_new ? k0 + INJ_PER_BLOCK : n_new;
    for (int64_t k = k0 + threadIdx.x; k < k_end; k += INJ_BLOCK) {
        const int64_t slot = base + k;
        if (slot >= T.capacity) continue;
        double x2 = 0;
        for (int a = 0; a < MAX_ATTEMPTS; ++a) {
            const U4 u = philox4x32_10(U4{stream_tag, (uint32_t)s | (P_INJ_POS << 8), (uint32_t)k,
                                          (uint32_t)a}, gp.key0, gp.key1);
            const double cx2 = -1.0 + 2.0 * unit_open(u.x);
            const double r = r_of(xo, cx2, alpha);
            const double t = alpha / (r + 2.0 * alpha * cx2);
            const double dA = 6.283185307179586 * r * r * sqrt(1.0 + (1.0 - cx2 * cx2) * t * t);
            if (unit_open(u.y) * gp.M_area <= dA || a == MAX_ATTEMPTS - 1) {
                x2 = cx2;
                break;
            }
        }
        const U4 v = philox4x32_10(U4{stream_tag, (uint32_t)s | (P_INJ_VEL << 8), (uint32_t)k, 0u},
                                   gp.key0, gp.key1);
        const double vn = sp.sigma * sqrt(-2.0 * log(unit_open(v.x)));
        const double g = sp.sigma * sqrt(-2.0 * log(unit_open(v.y)));
        const double ang = 6.283185307179586 * unit_open(v.z);
        const double t1 = g * cos(ang), t2 = g * sin(ang);
        const double frac = unit_open(v.w);
        const double r = r_of(xo, x2, alpha);
        const double sn = sqrt(fmax(1.0 - x2 * x2, 0.0));
        const Metric<double> m = metric_at(r, x2, sn, alpha);
        const double gn = sqrt(m.x1R * m.x1R + m.x1Z * m.x1Z);
        const double nR = -m.x1R / gn, nZ = -m.x1Z / gn;
        const double vR = vn * nR + t1 * nZ;
        const double vZ = vn * nZ - t1 * nR;
        const double vT = t2;
        double x1n, x2n, vRn, vTn;
        const int st = drift_and_bound64(gp, sp, s, ns, r * sn, r * x2, vR, vZ, vT,
                                         gp.step * frac, x1n, x2n, vRn, vTn, tally, tally_count);
        gbl(b.id)[slot] = id0 + (uint32_t)k;
        if (st != 0) {
            store_dead(split, b, slot);
            if (st == 1) ++n_abs; else ++n_esc;
            continue;
        }
        store_particle(gp, split, b, slot, x1n, x2n, vRn, vZ, vTn);
        if (dep) {
            if (split) {
                const int32_t c = gbl(static_cast<int32_t*>(b.pos0))[slot];
                const float f1 = gbl(static_cast<float*>(b.pos1))[slot];
                const float f2 = gbl(static_cast<float*>(b.pos2))[slot];
                const int i1 = cell_i1(c), i2 = cell_i2(c);
                const float w00 = (1.f - f1) * (1.f - f2), w10 = f1 * (1.f - f2);
                const float w01 = (1.f - f1) * f2, w11 = f1 * f2;
                if (i1 >= n1 - 2) {
                    const int q = 3 * i2 + (i1 - (n1 - 2));
                    atomicAdd(&wf[q], w00);
                    atomicAdd(&wf[q + 1], w10);
                    atomicAdd(&wf[q + 3], w01);
                    atomicAdd(&wf[q + 4], w11);
                } else {
                    float* d = static_cast<float*>(dep);
                    const int o = i2 * nx + i1;
                    gadd(&d[o], w00);
                    gadd(&d[o + 1], w10);
                    gadd(&d[o + nx], w01);
                    gadd(&d[o + nx + 1], w11);
                }
            } else {
                int i1, i2;
                double f1, f2;
                locate64(gp, x1n, x2n, i1, i2, f1, f2);
                const double w00 = (1 - f1) * (1 - f2), w10 = f1 * (1 - f2), w01 = (1 - f1) * f2, w11 = f1 * f2;
                if (i1 >= n1 - 2) {
                    const int q = 3 * i2 + (i1 - (n1 - 2));
                    atomicAdd(&wd[q], w00);
                    atomicAdd(&wd[q + 1], w10);
                    atomicAdd(&wd[q + 3], w01);
                    atomicAdd(&wd[q + 4], w11);
                } else {
                    double* d = static_cast<double*>(dep);
                    const int o = i2 * nx + i1;
                    gadd(&d[o], w00);
                    gadd(&d[o + 1], w10);
                    gadd(&d[o + nx], w01);
                    gadd(&d[o + nx + 1], w11);
                }
            }
        }
    }
    if (dep) {
        __syncthreads();
        for (int q = threadIdx.x; q < wn; q += INJ_BLOCK) {
            const int o = (q / 3) * nx + (n1 - 2) + q % 3;
            if (split) {
                const float v = wf[q];
                if (v != 0.f) gadd(&static_cast<float*>(dep)[o], v);
            } else {
                const double v = wd[q];
                if (v != 0.0) gadd(&static_cast<double*>(dep)[o], v);
            }
        }
    }
    block_count_add(n_abs, reinterpret_cast<unsigned long long*>(&ctr->absorbed[s]));
    block_count_add(n_esc, reinterpret_cast<unsigned long long*>(&ctr->escaped[s]));
}

// ----------------------------------------------------------------- readback
__global__ void __launch_bounds__(BLOCK)
k_readback(GrainParams gp, int s, bool split, PBuf b, const DevCounters* __restrict__ ctr,
           double* x1o, double* x2o, double* vRo, double* vZo, double* vTo, int64_t* ido,
           unsigned long long* cursor) {
    const int64_t n = ctr->n[s];
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        double x1, x2, vR, vZ, vT;
        if (split) {
            const int32_t c = gbl(static_cast<const int32_t*>(b.pos0))[p];
            if (c < 0) continue;
            x1 = -1.0 + ((double)cell_i1(c) + (double)gbl(static_cast<const float*>(b.pos1))[p]) * gp.h1;
            const double u = ((double)cell_i2(c) + (double)gbl(static_cast<const float*>(b.pos2))[p]) * gp.h2;
            x2 = -1.0 + u;
            vR = gbl(static_cast<const float*>(b.vR))[p];
            vZ = gbl(static_cast<const float*>(b.vZ))[p];
            vT = gbl(static_cast<const float*>(b.vT))[p];
        } else {
            x1 = gbl(static_cast<const double*>(b.pos1))[p];
            if (x1 > 0.0) continue;
            x2 = gbl(static_cast<const double*>(b.pos2))[p];
            vR = gbl(static_cast<const double*>(b.vR))[p];
            vZ = gbl(static_cast<const double*>(b.vZ))[p];
            vT = gbl(static_cast<const double*>(b.vT))[p];
        }
        const unsigned long long o = __hip_atomic_fetch_add(gbl(cursor), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x1o[o] = x1;
        x2o[o] = x2;
        vRo[o] = vR;
        vZo[o] = vZ;
        vTo[o] = vT;
        ido[o] = (int64_t)gbl(b.id)[p];
    }
}

// ----------------------------------------------------------------- tile sort
// Particles are ordered by tiles of 2^tile_log2 x 2^tile_log2 cells (tiles in
// row-major order, x1 fastest); inside a tile the order is arbitrary.  That is
// all the push needs: a chunk of consecutive particles then covers one tile (or
// a few), so its deposit window and its field nodes stay small.  The sort is a
// one-pass counting sort without global atomics, run for every task at once
// (blockIdx.y = task): each of the task's sort_blocks workgroups takes a
// contiguous slot range and builds the histogram of its tiles in LDS, the
// histograms are scanned tile-major, and each workgroup scatters its particles
// to its own offsets.  Dead slots are dropped on the way.
constexpr int SORT_BLOCKS_MAX = 1024;
constexpr int SCAN_SEG = 4096;      // histogram entries per scan workgroup

int max_sort_blocks() { return SORT_BLOCKS_MAX; }
int scan_seg_len() { return SCAN_SEG; }

__device__ inline int tile_of(const GrainParams& gp, int i1, int i2) {
    return (i2 >> gp.tile_log2) * gp.ntx + (i1 >> gp.tile_log2);
}

// One particle's slot contents, moved as a unit by the scatter; its tile key
// comes from the position words it already holds.
template <bool SPLIT> struct Moved;
template <> struct Moved<true> {
    uint32_t w[7];      // cell, f1, f2, vR, vZ, vT, id
};
template <> struct Moved<false> {
    uint64_t d[5];      // x1, x2, vR, vZ, vT bits
    uint32_t id;
};

__device__ inline int tile_key(const GrainParams& gp, const Moved<true>& m) {
    const int32_t c = (int32_t)m.w[0];
    if (c < 0) return -1;
    return tile_of(gp, cell_i1(c), cell_i2(c));
}
__device__ inline int tile_key(const GrainParams& gp, const Moved<false>& m) {
    const double x1 = __builtin_bit_cast(double, m.d[0]);
    if (x1 > 0.0) return -1;
    int i1, i2;
    double f1, f2;
    locate64(gp, x1, __builtin_bit_cast(double, m.d[1]), i1, i2, f1, f2);
    return tile_of(gp, i1, i2);
}

// the position words only (histogram pass)
__device__ inline void load_pos(const PBuf& b, int64_t p, Moved<true>& m) {
    m.w[0] = *slot4(static_cast<const uint32_t*>(b.pos0), p);
}
__device__ inline void load_pos(const PBuf& b, int64_t p, Moved<false>& m) {
    m.d[0] = gbl(static_cast<const uint64_t*>(b.pos1))[p];
    m.d[1] = gbl(static_cast<const uint64_t*>(b.pos2))[p];
}

__device__ inline void load_moved(const PBuf& b, int64_t p, Moved<true>& m) {
    m.w[0] = *slot4(static_cast<const uint32_t*>(b.pos0), p);
    m.w[1] = *slot4(static_cast<const uint32_t*>(b.pos1), p);
    m.w[2] = *slot4(static_cast<const uint32_t*>(b.pos2), p);
    m.w[3] = *slot4(static_cast<const uint32_t*>(b.vR), p);
    m.w[4] = *slot4(static_cast<const uint32_t*>(b.vZ), p);
    m.w[5] = *slot4(static_cast<const uint32_t*>(b.vT), p);
    m.w[6] = *slot4(static_cast<const uint32_t*>(b.id), p);
}
__device__ inline void load_moved(const PBuf& b, int64_t p, Moved<false>& m) {
    m.d[0] = gbl(static_cast<const uint64_t*>(b.pos1))[p];
    m.d[1] = gbl(static_cast<const uint64_t*>(b.pos2))[p];
    m.d[2] = gbl(static_cast<const uint64_t*>(b.vR))[p];
    m.d[3] = gbl(static_cast<const uint64_t*>(b.vZ))[p];
    m.d[4] = gbl(static_cast<const uint64_t*>(b.vT))[p];
    m.id = gbl(b.id)[p];
}

__device__ inline void store_moved(const PBuf& b, int64_t o, const Moved<true>& m) {
    *slot4(static_cast<uint32_t*>(b.pos0), o) = m.w[0];
    *slot4(static_cast<uint32_t*>(b.pos1), o) = m.w[1];
    *slot4(static_cast<uint32_t*>(b.pos2), o) = m.w[2];
    *slot4(static_cast<uint32_t*>(b.vR), o) = m.w[3];
    *slot4(static_cast<uint32_t*>(b.vZ), o) = m.w[4];
    *slot4(static_cast<uint32_t*>(b.vT), o) = m.w[5];
    *slot4(static_cast<uint32_t*>(b.id), o) = m.w[6];
}
__device__ inline void store_moved(const PBuf& b, int64_t o, const Moved<false>& m) {
    gbl(static_cast<uint64_t*>(b.pos1))[o] = m.d[0];
    gbl(static_cast<uint64_t*>(b.pos2))[o] = m.d[1];
    gbl(static_cast<uint64_t*>(b.vR))[o] = m.d[2];
    gbl(static_cast<uint64_t*>(b.vZ))[o] = m.d[3];
    gbl(static_cast<uint64_t*>(b.vT))[o] = m.d[4];
    gbl(b.id)[o] = m.id;
}

// Run-length segments of equal keys inside a wave (all 64 lanes active): the
// first lane of each run is its head; head_lane and, for heads, the run length.
__device__ inline void wave_runs(int key, int& head_lane, int& run_len, bool& is_head) {
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(key, 1);
    is_head = (lane == 0) || (key != prev);
    const unsigned long long hm = __ballot(is_head);
    const unsigned long long le = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1);
    head_lane = 63 - __clzll((long long)(hm & le));
    const unsigned long long gt = hm & ~le;
    run_len = (gt ? (__ffsll((long long)gt) - 1) : 64) - lane;
}

// A value read from memory the kernel also writes (a vector load) that is the
// same in every lane, moved to scalar registers: array bases selected by it are
// then scalar too, and no loop waits on the vector load that produced them.
__device__ inline int64_t uniform64(int64_t v) {
    return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
                     (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)v));
}

__device__ inline void sort_range(int64_t n, int blocks, int64_t& lo, int64_t& hi) {
    const int64_t per = (n + blocks - 1) / blocks;
    lo = min<int64_t>((int64_t)blockIdx.x * per, n);
    hi = min<int64_t>(lo + per, n);
}

// Batches of BLOCK slots per iteration of the histogram and scatter loops,
// all their loads issued before the first is used (the scatter loads the next
// batch while it ranks, stages and stores the current one), so a workgroup's
// slot range streams with many loads in flight.
constexpr int HIST_BATCHES = 8;
constexpr int SCATTER_BATCHES = 3;
static int scatter_batch() { return SCATTER_BATCHES * BLOCK; }

template <bool SPLIT>
__global__ void __launch_bounds__(BLOCK)
k_tile_hist(const PushTask* __restrict__ tasks, int max_level) {
    extern __shared__ int lh[];
    const PushTask& T = tasks[blockIdx.y];
    const int SB = T.sort_blocks;
    if ((int)blockIdx.x >= SB || T.sort_level > max_level) return;
    const GrainParams gp = T.gp;
    const int nt = gp.ntiles;
    for (int t = threadIdx.x; t < nt; t += BLOCK) lh[t] = 0;
    __syncthreads();
    const PBuf b = T.buf[__builtin_amdgcn_readfirstlane(T.ctr->cur[T.s])];
    int64_t lo, hi;
    sort_range(uniform64(T.ctr->n[T.s]), SB, lo, hi);
    for (int64_t base = lo; base < hi; base += HIST_BATCHES * BLOCK) {
        Moved<SPLIT> m[HIST_BATCHES];
        // every load is issued (a slot past the range reloads the last one):
        // loads behind a branch would each be waited for before the next
#pragma unroll
        for (int k = 0; k < HIST_BATCHES; ++k) {
            const int64_t p = base + k * BLOCK + threadIdx.x;
            load_pos(b, p < hi ? p : hi - 1, m[k]);
        }
#pragma unroll
        for (int k = 0; k < HIST_BATCHES; ++k) {
            const int64_t p = base + k * BLOCK + threadIdx.x;
            const int key = p < hi ? tile_key(gp, m[k]) : -1;
            int head, len;
            bool is_head;
            wave_runs(key, head, len, is_head);
            if (is_head && key >= 0) atomicAdd(&lh[key], len);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nt; t += BLOCK) gbl(T.hist)[(size_t)t * SB + blockIdx.x] = lh[t];
}

// Exclusive scan of every task's histogram (length ntiles * sort_blocks) in
// three passes: segment sums, scan of the segment sums (which also gives the
// live count), scan inside the segments.
__device__ inline int block_scan_excl(int v, int* tmp, int& total) {
    // exclusive scan of one int per thread over the block
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) tmp[w] = x;
    __syncthreads();
    int off = 0;
    total = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
        if (k < w) off += tmp[k];
        total += tmp[k];
    }
    __syncthreads();
    return off + x - v;
}

__global__ void __launch_bounds__(BLOCK)
k_scan_reduce(const PushTask* __restrict__ tasks, int max_level) {
    const PushTask& T = tasks[blockIdx.y];
    if (T.sort_level > max_level) return;
    const int64_t len = (int64_t)T.gp.ntiles * T.sort_blocks;
    const int64_t lo = (int64_t)blockIdx.x * SCAN_SEG;
    if (lo >= len) return;
    const int64_t hi = min<int64_t>(lo + SCAN_SEG, len);
    int v = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += BLOCK) v += gbl(T.hist)[i];
    __shared__ int tmp[BLOCK / 64];
    int total;
    (void)block_scan_excl(v, tmp, total);
    if (threadIdx.x == 0) gbl(T.seg)[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024)
k_scan_segs(const PushTask* __restrict__ tasks, int max_level) {
    const PushTask& T = tasks[blockIdx.x];
    if (T.sort_level > max_level) return;
    const int64_t len = (int64_t)T.gp.ntiles * T.sort_blocks;
    const int nseg = (int)((len + SCAN_SEG - 1) / SCAN_SEG);
    __shared__ int tmp[1024 / 64];
    int carry = 0;
    for (int k0 = 0; k0 < nseg; k0 += 1024) {
        const int k = k0 + threadIdx.x;
        const int v = k < nseg ? gbl(T.seg)[k] : 0;
        int total;
        const int ex = block_scan_excl(v, tmp, total);
        if (k < nseg) gbl(T.seg)[k] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        gbl(T.hist_off)[len] = carry;
        T.ctr->n_sorted[T.s] = carry;
    }
}

__global__ void __launch_bounds__(BLOCK)
k_scan_apply(const PushTask* __restrict__ tasks, int max_level) {
    const PushTask& T = tasks[blockIdx.y];
    if (T.sort_level > max_level) return;
    const int64_t len = (int64_t)T.gp.ntiles * T.sort_blocks;
    const int64_t lo = (int64_t)blockIdx.x * SCAN_SEG;
    if (lo >= len) return;
    constexpr int PER = SCAN_SEG / BLOCK;
    const int64_t i0 = lo + (int64_t)threadIdx.x * PER;
    int v[PER];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = (i0 + k < len) ? gbl(T.hist)[i0 + k] : 0;
        sum += v[k];
    }
    __shared__ int tmp[BLOCK / 64];
    int total;
    int run = gbl(T.seg)[blockIdx.x] + block_scan_excl(sum, tmp, total);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (i0 + k < len) gbl(T.hist_off)[i0 + k] = run;
        run += v[k];
    }
}

// 32-bit words of a moved slot, for staging in LDS.
template <bool SPLIT> struct Words;
template <> struct Words<true> {
    static constexpr int N = 7;
    static __device__ uint32_t get(const Moved<true>& m, int w) { return m.w[w]; }
    static __device__ void set(Moved<true>& m, int w, uint32_t v) { m.w[w] = v; }
};
template <> struct Words<false> {
    static constexpr int N = 11;
    static __device__ uint32_t get(const Moved<false>& m, int w) {
        return w < 10 ? (uint32_t)(m.d[w >> 1] >> (32 * (w & 1))) : m.id;
    }
    static __device__ void set(Moved<false>& m, int w, uint32_t v) {
        if (w == 10) {
            m.id = v;
        } else {
            const int sh = 32 * (w & 1);
            m.d[w >> 1] = (m.d[w >> 1] & ~(0xFFFFFFFFull << sh)) | ((uint64_t)v << sh);
        }
    }
};

// Scatter, one batch of SCATTER_BATCHES * BLOCK consecutive slots at a time:
// (1) every slot of the batch is loaded (all loads in flight together);
// (2) a per-tile LDS counter ranks each particle within its tile in the batch,
//     and the first particle of a tile enters the tile in the batch's list;
// (3) the list's counts are scanned, which orders the batch by tile, and each
//     tile takes its destination range from the workgroup's cursor;
// (4) the particles are staged in LDS in that order and written out by
//     consecutive threads to consecutive slots, so the stores of a wave form
//     whole cache lines instead of one partial line per particle.
// LDS: cursors and counters per tile (2 x ntiles ints), the batch's tile list
// (tile, count | first, destination), and the staged words and destinations.
template <bool SPLIT>
__global__ void __launch_bounds__(BLOCK)
k_tile_scatter(const PushTask* __restrict__ tasks, int max_level) {
    constexpr int B = SCATTER_BATCHES * BLOCK;
    constexpr int NW = Words<SPLIT>::N;
    extern __shared__ int lds_i[];
    __shared__ int nkeys, nlive;
    const PushTask& T = tasks[blockIdx.y];
    const int SB = T.sort_blocks;
    if ((int)blockIdx.x >= SB || T.sort_level > max_level) return;
    const GrainParams gp = T.gp;
    const int nt = gp.ntiles;
    int* cur = lds_i;                 // [ntiles] next destination slot of each tile
    int* cnt = cur + nt;              // [ntiles] batch count (low 16 bits) | list index + 1 (high bits)
    int* keys = cnt + nt;             // [B] the batch's tiles, in order of first appearance
    int* first = keys + B;            // [B] their first position in tile order
    int* dest = first + B;            // [B] their first destination slot
    uint32_t* stage = reinterpret_cast<uint32_t*>(dest + B);   // [NW + 1][B]
    for (int t = threadIdx.x; t < nt; t += BLOCK) {
        cur[t] = gbl(T.hist_off)[(size_t)t * SB + blockIdx.x];
        cnt[t] = 0;
    }
    if (threadIdx.x == 0) nkeys = 0;
    __syncthreads();
    const int which = __builtin_amdgcn_readfirstlane(T.ctr->cur[T.s]);
    const PBuf src = T.buf[which];
    const PBuf dst = T.buf[1 - which];
    int64_t lo, hi;
    sort_range(uniform64(T.ctr->n[T.s]), SB, lo, hi);
    if (lo >= hi) return;
    // every load is issued (a slot past the range reloads the last one); the
    // next batch is loaded while the current one is ranked, staged and stored
    Moved<SPLIT> m[SCATTER_BATCHES];
#pragma unroll
    for (int k = 0; k < SCATTER_BATCHES; ++k) {
        const int64_t p = lo + k * BLOCK + threadIdx.x;
        load_moved(src, p < hi ? p : hi - 1, m[k]);
    }
    for (int64_t base = lo; base < hi; base += B) {
        Moved<SPLIT> nx[SCATTER_BATCHES];
#pragma unroll
        for (int k = 0; k < SCATTER_BATCHES; ++k) {
            const int64_t p = base + B + k * BLOCK + threadIdx.x;
            load_moved(src, p < hi ? p : hi - 1, nx[k]);
        }
        int key[SCATTER_BATCHES], rank[SCATTER_BATCHES];
#pragma unroll
        for (int k = 0; k < SCATTER_BATCHES; ++k) {
            const int64_t p = base + k * BLOCK + threadIdx.x;
            key[k] = p < hi ? tile_key(gp, m[k]) : -1;
            rank[k] = 0;
            if (key[k] >= 0) {
                const int old = atomicAdd(&cnt[key[k]], 1);
                rank[k] = old & 0xFFFF;
                if (rank[k] == 0) {
                    const int idx = atomicAdd(&nkeys, 1);
                    keys[idx] = key[k];
                    atomicOr(&cnt[key[k]], (idx + 1) << 16);
                }
            }
        }
        __syncthreads();
        // scan of the listed tiles' counts (one wave); destinations from the cursors
        const int nk = nkeys;
        if (threadIdx.x < 64) {
            int run = 0;
            for (int i0 = 0; i0 < nk; i0 += 64) {
                const int i = i0 + (int)threadIdx.x;
                const int c = i < nk ? (cnt[keys[i]] & 0xFFFF) : 0;
                int x = c;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(x, o);
                    if ((int)threadIdx.x >= o) x += y;
                }
                if (i < nk) {
                    first[i] = run + x - c;
                    dest[i] = cur[keys[i]];
                    cur[keys[i]] += c;
                }
                run += __shfl(x, 63);
            }
            if (threadIdx.x == 0) nlive = run;
        }
        __syncthreads();
        // stage in tile order, each particle with its destination slot
#pragma unroll
        for (int k = 0; k < SCATTER_BATCHES; ++k) {
            if (key[k] < 0) continue;
            const int idx = (cnt[key[k]] >> 16) - 1;
            const int pos = first[idx] + rank[k];
#pragma unroll
            for (int w = 0; w < NW; ++w) stage[w * B + pos] = Words<SPLIT>::get(m[k], w);
            stage[NW * B + pos] = (uint32_t)(dest[idx] + rank[k]);
        }
        __syncthreads();
        // consecutive threads write consecutive staged particles
        const int live = nlive;
        for (int q = threadIdx.x; q < live; q += BLOCK) {
            Moved<SPLIT> mm;
#pragma unroll
            for (int w = 0; w < NW; ++w) Words<SPLIT>::set(mm, w, stage[w * B + q]);
            store_moved(dst, (int64_t)stage[NW * B + q], mm);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nk; i += BLOCK) cnt[keys[i]] = 0;
        if (threadIdx.x == 0) nkeys = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SCATTER_BATCHES; ++k) m[k] = nx[k];
    }
}

// the sorted buffer becomes the current one; slots = live particles
__global__ void __launch_bounds__(BLOCK)
k_sort_commit(const PushTask* __restrict__ tasks, int ntasks, int max_level) {
    for (int t = threadIdx.x; t < ntasks; t += BLOCK) {
        if (tasks[t].sort_level > max_level) continue;
        DevCounters* ctr = tasks[t].ctr;
        const int s = tasks[t].s;
        ctr->n[s] = ctr->n_sorted[s];
        ctr->cur[s] = 1 - ctr->cur[s];
    }
}

__global__ void __launch_bounds__(BLOCK)
k_count_live(int s, bool split, PBuf b, const DevCounters* __restrict__ ctr,
             unsigned long long* out) {
    const int64_t n = ctr->n[s];
    uint32_t live = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        if (split) live += gbl(static_cast<const int32_t*>(b.pos0))[p] >= 0;
        else live += !(gbl(static_cast<const double*>(b.pos1))[p] > 0.0);
    }
    block_count_add(live, out);
}

// ----------------------------------------------------------------- launchers
static int grid_for(apic_ctx* ctx, int64_t n) {
    const int64_t want = (n + BLOCK - 1) / BLOCK;
    const int64_t cap = (int64_t)ctx->num_cus * 16;
    return (int)(want < 1 ? 1 : (want > cap ? cap : want));
}

static bool is_split(apic_ctx* ctx) { return ctx->opts.precision == APIC_FP32_SPLIT; }

// Workgroups of a persistent launch: push_wg_per_cu per compute unit, at most
// what stays resident at once (a second round of workgroups would run alone
// after the first and leave the chip underfilled), a multiple of 8 (XCDs).
template <typename K>
static int persistent_grid(apic_ctx* ctx, K kernel, int nt) {
    int resident = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, kernel, nt, 0) != hipSuccess || resident < 1)
        resident = 1;
    const int per_cu = std::min(ctx->sched.push_wg_per_cu, resident);
    int g = ctx->num_cus * per_cu;
    g = g / 8 * 8;
    return g < 8 ? 8 : g;
}

int push_resident_per_cu(apic_ctx* ctx) {
    int resident = 0;
    if (ctx->opts.precision == APIC_FP32_SPLIT)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, k_push_split, PushTraits<true>::NT, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, k_push_plain, PushTraits<false>::NT, 0);
    return resident < 1 ? 1 : resident;
}

hipError_t launch_push(apic_ctx* ctx, bool deposit) {
    const bool split = is_split(ctx);
    hipLaunchKernelGGL(k_plan_chunks, dim3(1), dim3(BLOCK), 0, ctx->stream, ctx->tasks, ctx->ntasks,
                       (int64_t)push_chunk(split), ctx->chunk_prefix);
    if (split)
        hipLaunchKernelGGL(k_push_split, dim3(persistent_grid(ctx, k_push_split, PushTraits<true>::NT)), dim3(PushTraits<true>::NT), 0, ctx->stream,
                           ctx->tasks, ctx->chunk_prefix, ctx->ntasks, deposit ? 1 : 0);
    else
        hipLaunchKernelGGL(k_push_plain, dim3(persistent_grid(ctx, k_push_plain, PushTraits<false>::NT)), dim3(PushTraits<false>::NT), 0, ctx->stream,
                           ctx->tasks, ctx->chunk_prefix, ctx->ntasks, deposit ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_deposit(apic_ctx* ctx) {
    const bool split = is_split(ctx);
    hipLaunchKernelGGL(k_plan_chunks, dim3(1), dim3(BLOCK), 0, ctx->stream, ctx->tasks, ctx->ntasks,
                       (int64_t)push_chunk(split), ctx->chunk_prefix);
    if (split)
        hipLaunchKernelGGL(k_deposit<true>, dim3(persistent_grid(ctx, k_deposit<true>, PushTraits<true>::NT)), dim3(PushTraits<true>::NT), 0,
                           ctx->stream, ctx->tasks, ctx->chunk_prefix, ctx->ntasks);
    else
        hipLaunchKernelGGL(k_deposit<false>, dim3(persistent_grid(ctx, k_deposit<false>, PushTraits<false>::NT)), dim3(PushTraits<false>::NT), 0,
                           ctx->stream, ctx->tasks, ctx->chunk_prefix, ctx->ntasks);
    return hipGetLastError();
}

hipError_t launch_inject(apic_ctx* ctx, bool deposit) {
    hipLaunchKernelGGL(k_inject_plan, dim3(1), dim3(BLOCK), 0, ctx->stream, ctx->tasks, ctx->ntasks);
    if (ctx->inj_blocks > 0)
        hipLaunchKernelGGL(k_inject, dim3(ctx->inj_blocks), dim3(INJ_BLOCK),
                           3 * (size_t)(ctx->max_n2 + 1) * (is_split(ctx) ? sizeof(float) : sizeof(double)), ctx->stream, ctx->tasks,
                           ctx->inj_block_task, is_split(ctx), deposit ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_sort(apic_ctx* ctx, int first_task, int n_tasks, int max_level) {
    const bool split = is_split(ctx);
    const size_t lds = sizeof(int) * (size_t)ctx->max_ntiles;
    // scatter: cursors and counters per tile, the batch's tile list and its staged words
    const size_t lds_scatter = sizeof(int) * (2 * (size_t)ctx->max_ntiles + 3 * (size_t)scatter_batch()) +
                               sizeof(uint32_t) * (size_t)(split ? 8 : 12) * scatter_batch();
    const PushTask* t = ctx->tasks + first_task;
    const dim3 sgrid(ctx->max_sort_blocks, n_tasks);
    const dim3 cgrid(ctx->max_segs, n_tasks);
    if (split) hipLaunchKernelGGL(k_tile_hist<true>, sgrid, dim3(BLOCK), lds, ctx->stream, t, max_level);
    else hipLaunchKernelGGL(k_tile_hist<false>, sgrid, dim3(BLOCK), lds, ctx->stream, t, max_level);
    hipLaunchKernelGGL(k_scan_reduce, cgrid, dim3(BLOCK), 0, ctx->stream, t, max_level);
    hipLaunchKernelGGL(k_scan_segs, dim3(n_tasks), dim3(1024), 0, ctx->stream, t, max_level);
    hipLaunchKernelGGL(k_scan_apply, cgrid, dim3(BLOCK), 0, ctx->stream, t, max_level);
    if (split) hipLaunchKernelGGL(k_tile_scatter<true>, sgrid, dim3(BLOCK), lds_scatter, ctx->stream, t, max_level);
    else hipLaunchKernelGGL(k_tile_scatter<false>, sgrid, dim3(BLOCK), lds_scatter, ctx->stream, t, max_level);
    hipLaunchKernelGGL(k_sort_commit, dim3(1), dim3(BLOCK), 0, ctx->stream, t, n_tasks, max_level);
    return hipGetLastError();
}

hipError_t launch_load(apic_ctx* ctx, Grain& g, int s, int64_t n) {
    const PBuf& b = g.buf[s][g.cur[s]];
    hipLaunchKernelGGL(k_load, dim3(grid_for(ctx, n)), dim3(BLOCK), 0, ctx->stream, g.gp, g.sp[s],
                       s, n, is_split(ctx), b);
    return hipGetLastError();
}

hipError_t launch_set_particles(apic_ctx* ctx, Grain& g, int s, int64_t n, const double* dx1,
                                const double* dx2, const double* dvR, const double* dvZ,
                                const double* dvT, int* d_bad) {
    const PBuf& b = g.buf[s][g.cur[s]];
    hipLaunchKernelGGL(k_set, dim3(grid_for(ctx, n)), dim3(BLOCK), 0, ctx->stream, g.gp, n,
                       is_split(ctx), b, dx1, dx2, dvR, dvZ, dvT, d_bad);
    return hipGetLastError();
}

hipError_t launch_readback(apic_ctx* ctx, Grain& g, int s, int64_t n, double* dx1, double* dx2,
                           double* dvR, double* dvZ, double* dvT, int64_t* did) {
    unsigned long long* cursor = reinterpret_cast<unsigned long long*>(&g.ctr->cursor);
    hipError_t e = launch_fill(ctx, cursor, sizeof(unsigned long long));
    if (e != hipSuccess) return e;
    const PBuf& b = g.buf[s][g.cur[s]];
    hipLaunchKernelGGL(k_readback, dim3(grid_for(ctx, n)), dim3(BLOCK), 0, ctx->stream, g.gp, s,
                       is_split(ctx), b, g.ctr, dx1, dx2, dvR, dvZ, dvT, did, cursor);
    return hipGetLastError();
}

// ----------------------------------------------------------------- static scratch
// Staging of the allocation-free particle upload (apic_inject_noalloc): the
// host arrays of at most NOALLOC_MAX_PARTICLES particles as five FP64 columns
// (x1, x2, vR, vZ, vTheta), then one word for the out-of-domain flag.  A
// file-scope device array: every GPU the library runs on holds its own copy
// (10 MiB) until the process ends, and calls that overlap on one GPU race on
// it.  In host code `scratch` names a host-side stand-in, so its device
// address is looked up once per device and only that address is used.
static __device__ __align__(256) double scratch[5 * NOALLOC_MAX_PARTICLES + 32];

hipError_t noalloc_scratch(double** out) {
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static double* addr[MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double*>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_count_live(apic_ctx* ctx, Grain& g, int s, unsigned long long* out) {
    hipError_t e = launch_fill(ctx, out, sizeof(unsigned long long));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_count_live, dim3(grid_for(ctx, g.capacity[s])), dim3(BLOCK), 0,
                       ctx->stream, s, is_split(ctx), g.buf[s][g.cur[s]], g.ctr, out);
    return hipGetLastError();
}

}  // namespace apic
