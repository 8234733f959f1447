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
#include "apic_internal.h"
#include "device_common.h"

#include <hipcub/hipcub.hpp>

namespace apic {

constexpr int BLOCK = 256;
constexpr double FP64_DEAD = 1.0;   // x1 of a dead FP64 slot (valid x1 < 0)

__device__ inline void atomic_add_f64(double* p, double v) { atomicAdd(p, v); }

// Block-wide sum of a per-thread u32 followed by one atomic per block.
__device__ inline void block_count_add(uint32_t v, unsigned long long* dst) {
    __shared__ uint32_t red[BLOCK / 64];
    uint32_t w = v;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
        if (t) atomicAdd(dst, (unsigned long long)t);
    }
    __syncthreads();
}

// ----------------------------------------------------------------- impact tally
// Bisection on x1 + 1 along the chord P(t) = (R + t dX, t dY, Z + t dZ) between
// t = 0 (outside) and t_in (inside); tallies at the impact point with the
// velocity rotated into the impact point's meridional plane.
template <typename T>
__device__ void tally_impact(const GrainParams& gp, const SpeciesParams& sp, int s, int ns,
                             T R, T Z, T dX, T dY, T dZ, T t_in, T vR, T vZ, T vT,
                             double* tally, unsigned long long* tally_count, int iters) {
    const T alpha = (T)gp.alpha;
    T lo = 0, hi = t_in;
    for (int it = 0; it < iters; ++it) {
        const T mid = T(0.5) * (lo + hi);
        const T X = R + mid * dX, Y = mid * dY, Zc = Z + mid * dZ;
        const T r = sqrt(X * X + Y * Y + Zc * Zc);
        const T x1 = x1_of(r, Zc / r, alpha);
        const bool inside = !(x1 > T(-1));
        hi = inside ? mid : hi;
        lo = inside ? lo : mid;
    }
    const T X = R + hi * dX, Y = hi * dY, Zi = Z + hi * dZ;
    const T Ri = sqrt(X * X + Y * Y);
    const T ri = sqrt(Ri * Ri + Zi * Zi);
    const T x2 = Zi / ri;
    int b = (int)floor((x2 + T(1)) * T(0.5) * (T)gp.n_bins);
    b = b < 0 ? 0 : (b >= gp.n_bins ? gp.n_bins - 1 : b);
    T c = 1, sn = 0;
    if (Ri > T(0)) { c = X / Ri; sn = Y / Ri; }
    const double vRi = (double)(c * vR + sn * vT);
    const double vTi = (double)(-sn * vR + c * vT);
    const double v2 = (double)vR * vR + (double)vZ * vZ + (double)vT * vT;
    const size_t stride = (size_t)ns * gp.n_bins;
    const size_t o = (size_t)s * gp.n_bins + b;
    atomic_add_f64(&tally[o], sp.q * sp.w);
    atomic_add_f64(&tally[stride + o], sp.m * sp.w * vRi);
    atomic_add_f64(&tally[2 * stride + o], sp.m * sp.w * (double)vZ);
    atomic_add_f64(&tally[3 * stride + o], sp.m * sp.w * (double)Ri * vTi);
    atomic_add_f64(&tally[4 * stride + o], sp.w * (0.5 * sp.m * v2 + sp.e_bind));
    atomicAdd(&tally_count[o], 1ull);
}

// Closest approach of the chord to the origin; returns t in (0,1) if the point
// there is inside the grain, else -1.
template <typename T>
__device__ inline T chord_inside(const GrainParams& gp, T R, T Z, T dX, T dY, T dZ) {
    const T dd = dX * dX + dY * dY + dZ * dZ;
    if (!(dd > T(0))) return T(-1);
    const T tc = -(R * dX + Z * dZ) / dd;
    if (!(tc > T(0) && tc < T(1))) return T(-1);
    const T X = R + tc * dX, Y = tc * dY, Zc = Z + tc * dZ;
    const T rc2 = X * X + Y * Y + Zc * Zc;
    const T rg = (T)gp.r_grain_max;
    if (rc2 > rg * rg) return T(-1);
    const T rc = sqrt(rc2);
    const T x1 = x1_of(rc, Zc / rc, (T)gp.alpha);
    return (x1 > T(-1)) ? T(-1) : tc;
}

// ----------------------------------------------------------------- FP32 split push
__global__ void __launch_bounds__(BLOCK)
k_push_split(GrainParams gp, SpeciesParams sp, int s, int ns,
             int32_t* __restrict__ cell, float* __restrict__ f1a, float* __restrict__ f2a,
             float* __restrict__ vRa, float* __restrict__ vZa, float* __restrict__ vTa,
             const float2* __restrict__ grad, float* __restrict__ dep,
             DevCounters* __restrict__ ctr, double* __restrict__ tally,
             unsigned long long* __restrict__ tally_count) {
    const int64_t n = ctr->n[s];
    const int n1 = gp.n1, n2 = gp.n2, nx = gp.nx;
    const float alpha = (float)gp.alpha;
    const float h1 = (float)gp.h1, h2 = (float)gp.h2;
    const float ih1 = (float)gp.inv_h1, ih2 = (float)gp.inv_h2;
    const float mx1_out = (float)(-gp.x1_out);
    const float step = (float)gp.step;
    const float qmh = (float)sp.qm_half;
    const float rcm1 = (float)sp.rot_cm1, rs = (float)sp.rot_s;
    uint32_t n_live = 0, n_abs = 0, n_esc = 0;

    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = cell[p];
        if (c < 0) continue;
        ++n_live;
        const int i1 = cell_i1(c), i2 = cell_i2(c);
        const float f1 = f1a[p], f2 = f2a[p];
        float vR = vRa[p], vZ = vZa[p], vT = vTa[p];

        // gather (bilinear in the logical coordinates)
        const int idx = i2 * nx + i1;
        const float2 g00 = grad[idx], g10 = grad[idx + 1];
        const float2 g01 = grad[idx + nx], g11 = grad[idx + nx + 1];
        const float e1 = 1.f - f1, e2 = 1.f - f2;
        const float w00 = e1 * e2, w10 = f1 * e2, w01 = e1 * f2, w11 = f1 * f2;
        const float p1 = w00 * g00.x + w10 * g10.x + w01 * g01.x + w11 * g11.x;
        const float p2 = w00 * g00.y + w10 * g10.y + w01 * g01.y + w11 * g11.y;

        // geometry at the particle from the cell index: -x1 measured from the
        // outer boundary (no cancellation where |x1| is small), 1 + x2 and 1 - x2
        // measured from the two axis ends
        const float x1 = -(mx1_out + ((float)(n1 - i1) - f1) * h1);
        const float opx2 = ((float)i2 + f2) * h2;
        const float omx2 = ((float)(n2 - i2) - f2) * h2;
        const float x2 = 0.5f * (opx2 - omx2);
        const float sn = sqrtf(opx2 * omx2);
        const float r = r_of(x1, x2, alpha);
        const float R = r * sn, Z = r * x2;
        const Metric<float> m = metric_at(r, x2, sn, alpha);
        const float ER = -(m.x1R * p1 + m.x2R * p2);
        const float EZ = -(m.x1Z * p1 + m.x2Z * p2);

        // Boris kick (eq. 9: dV_R = -omega V_Theta dt, dV_Theta = +omega V_R dt).
        // The rotation is applied as v + ((cos - 1) v + sin v_perp) with cos - 1
        // held separately, so its FP32 form preserves |v| to ~1e-10 per step
        // instead of drifting by the rounding of cos.
        vR += qmh * ER;
        vZ += qmh * EZ;
        {
            const float t = vR + (rcm1 * vR - rs * vT);
            vT = vT + (rs * vR + rcm1 * vT);
            vR = t;
        }
        vR += qmh * ER;
        vZ += qmh * EZ;

        // drift in the local Cartesian frame
        const float dX = step * vR, dY = step * vT, dZ = step * vZ;
        const float X = R + dX, Zn = Z + dZ;
        const float Rn2 = X * X + dY * dY;
        const float Rn = sqrtf(Rn2);
        // rotation of (v_R, v_Theta) into the new meridional plane, again as
        // v + ((cos - 1) v + sin v_perp) with cos - 1 = -dY^2 / (R' (X + R'))
        float cm = 0.f, sr = 0.f;
        if (Rn > 0.f) {
            const float iR = 1.f / Rn;
            sr = dY * iR;
            cm = X > 0.f ? -(dY * dY) * iR / (X + Rn) : X * iR - 1.f;
        }
        const float vRn = vR + (cm * vR + sr * vT);
        const float vTn = vT + (-sr * vR + cm * vT);

        // new conforming position from the displacement
        const float dr2 = 2.f * (R * dX + Z * dZ) + (dX * dX + dY * dY + dZ * dZ);  // r'^2 - r^2
        const float rn = sqrtf(Rn2 + Zn * Zn);
        const float dr = dr2 / (rn + r);
        const float irr = 1.f / (r * rn);
        const float dx2 = (dZ * r - Z * dr) * irr;
        const float dx1 = dr * irr - alpha * (dx2 * r * r - x2 * dr * (2.f * r + dr)) * irr * irr;
        float t1 = f1 + dx1 * ih1;
        float k1 = floorf(t1);
        int i1n = i1 + (int)k1;
        float f1n = t1 - k1;
        if (f1n >= 1.f) { f1n = 0.f; ++i1n; }
        float t2 = f2 + dx2 * ih2;
        float k2 = floorf(t2);
        int i2n = i2 + (int)k2;
        float f2n = t2 - k2;
        if (f2n >= 1.f) { f2n = 0.f; ++i2n; }
        if (i2n <= 0 || i2n >= n2 - 1) {
            // next to the axis: distance to it from 1 -+ x2' = R'^2 / (r' (r' +- Z'))
            if (Zn > 0.f) {
                const float u = Rn2 / (rn * (rn + Zn)) * ih2;     // (1 - x2') / h2
                const float j = floorf(u);
                i2n = n2 - 1 - (int)j;
                f2n = 1.f - (u - j);
                if (f2n >= 1.f) { f2n = 0.f; ++i2n; }
            } else {
                const float u = Rn2 / (rn * (rn - Zn)) * ih2;     // (1 + x2') / h2
                const float j = floorf(u);
                i2n = (int)j;
                f2n = u - j;
            }
            if (i2n < 0) { i2n = 0; f2n = 0.f; }
            if (i2n > n2 - 1) { i2n = n2 - 1; f2n = 0.99999994f; }
        }

        // boundaries
        const float tmid = chord_inside<float>(gp, R, Z, dX, dY, dZ);
        if (i1n < 0 || tmid > 0.f) {
            const float t_in = tmid > 0.f ? tmid : 1.f;
            tally_impact<float>(gp, sp, s, ns, R, Z, dX, dY, dZ, t_in, vR, vZ, vT, tally,
                                tally_count, 24);
            cell[p] = DEAD;
            ++n_abs;
            continue;
        }
        if (i1n >= n1) {
            cell[p] = DEAD;
            ++n_esc;
            continue;
        }
        cell[p] = pack_cell(i1n, i2n);
        f1a[p] = f1n;
        f2a[p] = f2n;
        vRa[p] = vRn;
        vZa[p] = vZ;
        vTa[p] = vTn;
        if (dep) {
            const int o = i2n * nx + i1n;
            const float a1 = 1.f - f1n, a2 = 1.f - f2n;
            atomicAdd(&dep[o], a1 * a2);
            atomicAdd(&dep[o + 1], f1n * a2);
            atomicAdd(&dep[o + nx], a1 * f2n);
            atomicAdd(&dep[o + nx + 1], f1n * f2n);
        }
    }
    block_count_add(n_live, reinterpret_cast<unsigned long long*>(&ctr->pushed[s]));
    block_count_add(n_abs, reinterpret_cast<unsigned long long*>(&ctr->absorbed[s]));
    block_count_add(n_esc, reinterpret_cast<unsigned long long*>(&ctr->escaped[s]));
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
    atomicAdd(&dep[o], (1 - f1) * (1 - f2));
    atomicAdd(&dep[o + 1], f1 * (1 - f2));
    atomicAdd(&dep[o + gp.nx], (1 - f1) * f2);
    atomicAdd(&dep[o + gp.nx + 1], f1 * f2);
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
    const double tmid = chord_inside<double>(gp, R, Z, dX, dY, dZ);
    if (!(x1n > -1.0) || tmid > 0.0) {
        tally_impact<double>(gp, sp, s, ns, R, Z, dX, dY, dZ, tmid > 0.0 ? tmid : 1.0, vR, vZ,
                             vT, tally, tally_count, 48);
        return 1;
    }
    if (x1n >= gp.x1_out) return 2;
    return 0;
}

__global__ void __launch_bounds__(BLOCK)
k_push_plain(GrainParams gp, SpeciesParams sp, int s, int ns,
             double* __restrict__ x1a, double* __restrict__ x2a, double* __restrict__ vRa,
             double* __restrict__ vZa, double* __restrict__ vTa,
             const double2* __restrict__ grad, double* __restrict__ dep,
             DevCounters* __restrict__ ctr, double* __restrict__ tally,
             unsigned long long* __restrict__ tally_count) {
    const int64_t n = ctr->n[s];
    const int nx = gp.nx;
    const double alpha = gp.alpha;
    uint32_t n_live = 0, n_abs = 0, n_esc = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const double x1 = x1a[p];
        if (x1 > 0.0) continue;
        ++n_live;
        const double x2 = x2a[p];
        double vR = vRa[p], vZ = vZa[p], vT = vTa[p];
        int i1, i2;
        double f1, f2;
        locate64(gp, x1, x2, i1, i2, f1, f2);
        const int idx = i2 * nx + i1;
        const double2 g00 = grad[idx], g10 = grad[idx + 1];
        const double2 g01 = grad[idx + nx], g11 = grad[idx + nx + 1];
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
        const int st = drift_and_bound64(gp, sp, s, ns, R, Z, vR, vZ, vT, gp.step, x1n, x2n, vRn,
                                         vTn, tally, tally_count);
        if (st != 0) {
            x1a[p] = FP64_DEAD;
            if (st == 1) ++n_abs; else ++n_esc;
            continue;
        }
        x1a[p] = x1n;
        x2a[p] = x2n;
        vRa[p] = vRn;
        vZa[p] = vZ;
        vTa[p] = vTn;
        if (dep) deposit64(gp, dep, x1n, x2n);
    }
    block_count_add(n_live, reinterpret_cast<unsigned long long*>(&ctr->pushed[s]));
    block_count_add(n_abs, reinterpret_cast<unsigned long long*>(&ctr->absorbed[s]));
    block_count_add(n_esc, reinterpret_cast<unsigned long long*>(&ctr->escaped[s]));
}

// ----------------------------------------------------------------- deposit only
__global__ void __launch_bounds__(BLOCK)
k_deposit_split(GrainParams gp, int s, const int32_t* __restrict__ cell,
                const float* __restrict__ f1a, const float* __restrict__ f2a,
                float* __restrict__ dep, const DevCounters* __restrict__ ctr) {
    const int64_t n = ctr->n[s];
    const int nx = gp.nx;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = cell[p];
        if (c < 0) continue;
        const int o = cell_i2(c) * nx + cell_i1(c);
        const float f1 = f1a[p], f2 = f2a[p];
        atomicAdd(&dep[o], (1.f - f1) * (1.f - f2));
        atomicAdd(&dep[o + 1], f1 * (1.f - f2));
        atomicAdd(&dep[o + nx], (1.f - f1) * f2);
        atomicAdd(&dep[o + nx + 1], f1 * f2);
    }
}

__global__ void __launch_bounds__(BLOCK)
k_deposit_plain(GrainParams gp, int s, const double* __restrict__ x1a,
                const double* __restrict__ x2a, double* __restrict__ dep,
                const DevCounters* __restrict__ ctr) {
    const int64_t n = ctr->n[s];
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const double x1 = x1a[p];
        if (x1 > 0.0) continue;
        deposit64(gp, dep, x1, x2a[p]);
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
        static_cast<int32_t*>(b.pos0)[p] = pack_cell(i1, i2);
        static_cast<float*>(b.pos1)[p] = ff1;
        static_cast<float*>(b.pos2)[p] = ff2;
        static_cast<float*>(b.vR)[p] = (float)vR;
        static_cast<float*>(b.vZ)[p] = (float)vZ;
        static_cast<float*>(b.vT)[p] = (float)vT;
    } else {
        static_cast<double*>(b.pos1)[p] = x1;
        static_cast<double*>(b.pos2)[p] = x2;
        static_cast<double*>(b.vR)[p] = vR;
        static_cast<double*>(b.vZ)[p] = vZ;
        static_cast<double*>(b.vT)[p] = vT;
    }
}

__device__ inline void store_dead(bool split, const PBuf& b, int64_t p) {
    if (split) static_cast<int32_t*>(b.pos0)[p] = DEAD;
    else static_cast<double*>(b.pos1)[p] = FP64_DEAD;
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
        b.id[k] = (uint32_t)k;
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
            atomicOr(bad, 1);
            store_dead(split, b, k);
        } else {
            store_particle(gp, split, b, k, a, c, vR[k], vZ[k], vT[k]);
        }
        b.id[k] = (uint32_t)k;
    }
}

// ----------------------------------------------------------------- injection
// Flux-Maxwellian injection at x1_out: x2 with density proportional to eq. (4),
// inward normal speed Rayleigh(sigma), tangential normal(0, sigma^2), then a
// straight partial step U * dt with the usual boundary tests; the survivors
// deposit their charge.  Slot = n_slots + k, id = next_id + k.
__global__ void __launch_bounds__(BLOCK)
k_inject(GrainParams gp, SpeciesParams sp, int s, int ns, int64_t n_new, uint32_t stream_tag,
         int64_t capacity, bool split, PBuf b, void* dep, DevCounters* ctr, double* tally,
         unsigned long long* tally_count) {
    const int64_t base = ctr->n[s];
    const uint32_t id0 = ctr->next_id[s];
    const double alpha = gp.alpha, xo = gp.x1_out;
    uint32_t n_abs = 0, n_esc = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_new;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t slot = base + k;
        if (slot >= capacity) {
            atomicOr(&ctr->overflow, 1u);
            continue;
        }
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
        b.id[slot] = id0 + (uint32_t)k;
        if (st != 0) {
            store_dead(split, b, slot);
            if (st == 1) ++n_abs; else ++n_esc;
            continue;
        }
        store_particle(gp, split, b, slot, x1n, x2n, vRn, vZ, vTn);
        if (dep) {
            if (split) {
                const int32_t c = static_cast<int32_t*>(b.pos0)[slot];
                const float f1 = static_cast<float*>(b.pos1)[slot];
                const float f2 = static_cast<float*>(b.pos2)[slot];
                float* d = static_cast<float*>(dep);
                const int o = cell_i2(c) * gp.nx + cell_i1(c);
                atomicAdd(&d[o], (1.f - f1) * (1.f - f2));
                atomicAdd(&d[o + 1], f1 * (1.f - f2));
                atomicAdd(&d[o + gp.nx], (1.f - f1) * f2);
                atomicAdd(&d[o + gp.nx + 1], f1 * f2);
            } else {
                deposit64(gp, static_cast<double*>(dep), x1n, x2n);
            }
        }
    }
    block_count_add(n_abs, reinterpret_cast<unsigned long long*>(&ctr->absorbed[s]));
    block_count_add(n_esc, reinterpret_cast<unsigned long long*>(&ctr->escaped[s]));
}

__global__ void k_add_slots(DevCounters* ctr, int s, int64_t n_new, int64_t capacity) {
    const int64_t n = ctr->n[s];
    const int64_t placed = (n + n_new > capacity) ? (capacity > n ? capacity - n : 0) : n_new;
    ctr->n[s] = n + placed;
    ctr->injected[s] += (uint64_t)placed;
    ctr->next_id[s] += (uint32_t)n_new;
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
            const int32_t c = static_cast<const int32_t*>(b.pos0)[p];
            if (c < 0) continue;
            x1 = -1.0 + ((double)cell_i1(c) + (double)static_cast<const float*>(b.pos1)[p]) * gp.h1;
            const double u = ((double)cell_i2(c) + (double)static_cast<const float*>(b.pos2)[p]) * gp.h2;
            x2 = -1.0 + u;
            vR = static_cast<const float*>(b.vR)[p];
            vZ = static_cast<const float*>(b.vZ)[p];
            vT = static_cast<const float*>(b.vT)[p];
        } else {
            x1 = static_cast<const double*>(b.pos1)[p];
            if (x1 > 0.0) continue;
            x2 = static_cast<const double*>(b.pos2)[p];
            vR = static_cast<const double*>(b.vR)[p];
            vZ = static_cast<const double*>(b.vZ)[p];
            vT = static_cast<const double*>(b.vT)[p];
        }
        const unsigned long long o = atomicAdd(cursor, 1ull);
        x1o[o] = x1;
        x2o[o] = x2;
        vRo[o] = vR;
        vZo[o] = vZ;
        vTo[o] = vT;
        ido[o] = (int64_t)b.id[p];
    }
}

// ----------------------------------------------------------------- counting sort
__device__ inline int sort_key(const GrainParams& gp, bool split, const PBuf& b, int64_t p,
                               int ncells) {
    if (split) {
        const int32_t c = static_cast<const int32_t*>(b.pos0)[p];
        return c < 0 ? ncells : cell_i2(c) * gp.n1 + cell_i1(c);
    }
    const double x1 = static_cast<const double*>(b.pos1)[p];
    if (x1 > 0.0) return ncells;
    int i1, i2;
    double f1, f2;
    locate64(gp, x1, static_cast<const double*>(b.pos2)[p], i1, i2, f1, f2);
    return i2 * gp.n1 + i1;
}

__global__ void __launch_bounds__(BLOCK)
k_sort_hist(GrainParams gp, int s, bool split, PBuf b, const DevCounters* __restrict__ ctr,
            int* __restrict__ count, int ncells) {
    const int64_t n = ctr->n[s];
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&count[sort_key(gp, split, b, p, ncells)], 1);
}

__global__ void __launch_bounds__(BLOCK)
k_sort_scatter(GrainParams gp, int s, bool split, PBuf src, PBuf dst,
               const DevCounters* __restrict__ ctr, int* __restrict__ cursor, int ncells) {
    const int64_t n = ctr->n[s];
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int key = sort_key(gp, split, src, p, ncells);
        if (key == ncells) continue;
        const int64_t o = atomicAdd(&cursor[key], 1);
        if (split) {
            static_cast<int32_t*>(dst.pos0)[o] = static_cast<const int32_t*>(src.pos0)[p];
            static_cast<float*>(dst.pos1)[o] = static_cast<const float*>(src.pos1)[p];
            static_cast<float*>(dst.pos2)[o] = static_cast<const float*>(src.pos2)[p];
            static_cast<float*>(dst.vR)[o] = static_cast<const float*>(src.vR)[p];
            static_cast<float*>(dst.vZ)[o] = static_cast<const float*>(src.vZ)[p];
            static_cast<float*>(dst.vT)[o] = static_cast<const float*>(src.vT)[p];
        } else {
            static_cast<double*>(dst.pos1)[o] = static_cast<const double*>(src.pos1)[p];
            static_cast<double*>(dst.pos2)[o] = static_cast<const double*>(src.pos2)[p];
            static_cast<double*>(dst.vR)[o] = static_cast<const double*>(src.vR)[p];
            static_cast<double*>(dst.vZ)[o] = static_cast<const double*>(src.vZ)[p];
            static_cast<double*>(dst.vT)[o] = static_cast<const double*>(src.vT)[p];
        }
        dst.id[o] = src.id[p];
    }
}

__global__ void k_sort_live(DevCounters* ctr, int s, const int* offset, int ncells) {
    ctr->n_sorted[s] = offset[ncells];
}

__global__ void k_sort_commit(DevCounters* ctr, int s) { ctr->n[s] = ctr->n_sorted[s]; }

// ----------------------------------------------------------------- launchers
static int grid_for(apic_ctx* ctx, int64_t n) {
    const int64_t want = (n + BLOCK - 1) / BLOCK;
    const int64_t cap = (int64_t)ctx->num_cus * 16;
    return (int)(want < 1 ? 1 : (want > cap ? cap : want));
}

static bool is_split(apic_ctx* ctx) { return ctx->opts.precision == APIC_FP32_SPLIT; }

hipError_t launch_push(apic_ctx* ctx, Grain& g, int s) {
    const PBuf& b = g.buf[s][g.cur[s]];
    const int grid = grid_for(ctx, g.host_slots[s]);
    void* dep = ctx->opts.frozen_field ? nullptr : g.dep[s];
    if (is_split(ctx)) {
        hipLaunchKernelGGL(k_push_split, dim3(grid), dim3(BLOCK), 0, ctx->stream, g.gp, g.sp[s], s,
                           g.ns, static_cast<int32_t*>(b.pos0), static_cast<float*>(b.pos1),
                           static_cast<float*>(b.pos2), static_cast<float*>(b.vR),
                           static_cast<float*>(b.vZ), static_cast<float*>(b.vT),
                           static_cast<const float2*>(g.grad), static_cast<float*>(dep), g.ctr,
                           g.tally, g.tally_count);
    } else {
        hipLaunchKernelGGL(k_push_plain, dim3(grid), dim3(BLOCK), 0, ctx->stream, g.gp, g.sp[s], s,
                           g.ns, static_cast<double*>(b.pos1), static_cast<double*>(b.pos2),
                           static_cast<double*>(b.vR), static_cast<double*>(b.vZ),
                           static_cast<double*>(b.vT), static_cast<const double2*>(g.grad),
                           static_cast<double*>(dep), g.ctr, g.tally, g.tally_count);
    }
    return hipGetLastError();
}

hipError_t launch_deposit_all(apic_ctx* ctx, Grain& g, int s) {
    const PBuf& b = g.buf[s][g.cur[s]];
    const int grid = grid_for(ctx, g.host_slots[s]);
    if (is_split(ctx))
        hipLaunchKernelGGL(k_deposit_split, dim3(grid), dim3(BLOCK), 0, ctx->stream, g.gp, s,
                           static_cast<const int32_t*>(b.pos0), static_cast<const float*>(b.pos1),
                           static_cast<const float*>(b.pos2), static_cast<float*>(g.dep[s]),
                           g.ctr);
    else
        hipLaunchKernelGGL(k_deposit_plain, dim3(grid), dim3(BLOCK), 0, ctx->stream, g.gp, s,
                           static_cast<const double*>(b.pos1), static_cast<const double*>(b.pos2),
                           static_cast<double*>(g.dep[s]), g.ctr);
    return hipGetLastError();
}

hipError_t launch_inject(apic_ctx* ctx, Grain& g, int s, int64_t n_new, uint32_t stream_tag) {
    const PBuf& b = g.buf[s][g.cur[s]];
    void* dep = ctx->opts.frozen_field ? nullptr : g.dep[s];
    hipLaunchKernelGGL(k_inject, dim3(grid_for(ctx, n_new)), dim3(BLOCK), 0, ctx->stream, g.gp,
                       g.sp[s], s, g.ns, n_new, stream_tag, g.capacity[s], is_split(ctx), b, dep,
                       g.ctr, g.tally, g.tally_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_add_slots(ctx, g, s, n_new);
}

hipError_t launch_add_slots(apic_ctx* ctx, Grain& g, int s, int64_t n_new) {
    hipLaunchKernelGGL(k_add_slots, dim3(1), dim3(1), 0, ctx->stream, g.ctr, s, n_new,
                       g.capacity[s]);
    g.host_slots[s] = std::min<int64_t>(g.host_slots[s] + n_new, g.capacity[s]);
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

hipError_t launch_sort(apic_ctx* ctx, Grain& g, int s) {
    const int nc = g.ncells;
    const PBuf& src = g.buf[s][g.cur[s]];
    const PBuf& dst = g.buf[s][1 - g.cur[s]];
    const int grid = grid_for(ctx, g.host_slots[s]);
    hipError_t e = launch_fill(ctx, g.sort_count, sizeof(int) * (size_t)(nc + 1));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_hist, dim3(grid), dim3(BLOCK), 0, ctx->stream, g.gp, s, is_split(ctx),
                       src, g.ctr, g.sort_count, nc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    size_t bytes = g.scan_tmp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(g.scan_tmp, bytes, g.sort_count, g.sort_offset, nc + 1,
                                         ctx->stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_live, dim3(1), dim3(1), 0, ctx->stream, g.ctr, s, g.sort_offset, nc);
    hipLaunchKernelGGL(k_sort_scatter, dim3(grid), dim3(BLOCK), 0, ctx->stream, g.gp, s,
                       is_split(ctx), src, dst, g.ctr, g.sort_offset, nc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_commit, dim3(1), dim3(1), 0, ctx->stream, g.ctr, s);
    g.cur[s] = 1 - g.cur[s];
    return hipGetLastError();
}

size_t scan_temp_bytes(int n) {
    size_t bytes = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (int*)nullptr, (int*)nullptr, n);
    return bytes;
}

}  // namespace apic

namespace apic {

__global__ void __launch_bounds__(BLOCK)
k_count_live(int s, bool split, PBuf b, const DevCounters* __restrict__ ctr,
             unsigned long long* out) {
    const int64_t n = ctr->n[s];
    uint32_t live = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        if (split) live += static_cast<const int32_t*>(b.pos0)[p] >= 0;
        else live += !(static_cast<const double*>(b.pos1)[p] > 0.0);
    }
    block_count_add(live, out);
}

hipError_t launch_count_live(apic_ctx* ctx, Grain& g, int s, unsigned long long* out) {
    hipError_t e = launch_fill(ctx, out, sizeof(unsigned long long));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_count_live, dim3(grid_for(ctx, g.host_slots[s])), dim3(BLOCK), 0,
                       ctx->stream, s, is_split(ctx), g.buf[s][g.cur[s]], g.ctr, out);
    return hipGetLastError();
}

}  // namespace apic
