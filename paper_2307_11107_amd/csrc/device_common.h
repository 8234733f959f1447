// Device-side helpers shared by the HIP kernels of the particle loop:
// Philox4x32-10, the conforming-coordinate geometry of eqs. (2), (3), (8) and
// the analytic coordinate derivatives used in eq. (10).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apic {

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): ten rounds of the 4x32 multiply-xor bijection with Weyl key bumps.
struct U4 { uint32_t x, y, z, w; };

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c.x;
        const uint64_t p1 = (uint64_t)M1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// u32 -> double in (0, 1)
__host__ __device__ inline double unit_open(uint32_t u) {
    return ((double)u + 0.5) * (1.0 / 4294967296.0);
}

// Philox stream tags and purposes (counter word 1 = species | purpose << 8)
constexpr uint32_t LOAD_STREAM = 0xFFFFFFFFu;
constexpr uint32_t P_LOAD_POS = 1, P_LOAD_VEL = 2, P_INJ_POS = 3, P_INJ_VEL = 4;
constexpr int MAX_ATTEMPTS = 64;

// ---------------------------------------------------------------- geometry
// eq. (3): r(x1, x2) = -(1 + sqrt(1 - 4 alpha x1 x2)) / (2 x1)
template <typename T>
__host__ __device__ inline T r_of(T x1, T x2, T alpha) {
    return -(T(1) + sqrt(T(1) - T(4) * alpha * x1 * x2)) / (T(2) * x1);
}

// eq. (2): x1(r, x2) = -(1/r)(1 + alpha x2 / r)
template <typename T>
__host__ __device__ inline T x1_of(T r, T x2, T alpha) {
    return -(T(1) + alpha * x2 / r) / r;
}

// Analytic derivatives of (x1, x2) with respect to (R, Z) at (r, x2), with
// s = sqrt(1 - x2^2) (chain rule through eqs. 2 and 8).
template <typename T>
struct Metric { T x1R, x1Z, x2R, x2Z; };

template <typename T>
__host__ __device__ inline Metric<T> metric_at(T r, T x2, T s, T alpha) {
    const T ir = T(1) / r;
    const T ir3 = ir * ir * ir;
    Metric<T> m;
    m.x1R = s * (r + T(3) * alpha * x2) * ir3;
    m.x1Z = (x2 * r + alpha * (T(3) * x2 * x2 - T(1))) * ir3;
    m.x2R = -x2 * s * ir;
    m.x2Z = s * s * ir;
    return m;
}

// Packed cell index of the FP32 split representation: (i2 << 16) | i1.
constexpr int32_t DEAD = -1;
__host__ __device__ inline int32_t pack_cell(int i1, int i2) { return (i2 << 16) | i1; }
__host__ __device__ inline int cell_i1(int32_t c) { return c & 0xFFFF; }
__host__ __device__ inline int cell_i2(int32_t c) { return (int)((uint32_t)c >> 16); }

}  // namespace apic

namespace apic {

// ---------------------------------------------------------------- global memory
// Pointers taken from descriptor tables in device memory are generic to the
// compiler, which then emits flat instructions (slower, and counted against
// the LDS wait counter too).  gbl() states that a pointer is global memory.
template <typename T>
using gptr = T __attribute__((address_space(1)))*;

template <typename T>
__device__ __forceinline__ gptr<T> gbl(T* p) { return (gptr<T>)p; }

__device__ __forceinline__ void gadd(float* p, float v) {
    __hip_atomic_fetch_add(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gadd(double* p, double v) {
    __hip_atomic_fetch_add(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gadd(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_add(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace apic
