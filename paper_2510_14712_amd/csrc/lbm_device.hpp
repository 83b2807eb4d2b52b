// Device-side building blocks of the non-ideal DDF lattice Boltzmann step
// (arXiv 2510.14712, Section 3.2): velocity set, product-form factors,
// van der Waals closed forms, boundary index rules and the population codec.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ---------------------------------------------------------------------------
// Velocity set: i = (c_x+1) + 3 (c_y+1) [+ 9 (c_z+1)]  (eq. D3Q27c)
// ---------------------------------------------------------------------------
template <int D> struct Lattice {
    static constexpr int Q = D == 2 ? 9 : 27;
    static constexpr int REST = D == 2 ? 4 : 13;
};
__host__ __device__ constexpr int cx_of(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy_of(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz_of(int i) { return i / 9 - 1; }
template <int D> __host__ __device__ constexpr int c_of(int i, int a) {
    return a == 0 ? cx_of(i) : (a == 1 ? cy_of(i) : (D == 3 ? cz_of(i) : 0));
}
template <int D> __host__ __device__ constexpr int csq_of(int i) {
    return cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + (D == 3 ? cz_of(i) * cz_of(i) : 0);
}

// ---------------------------------------------------------------------------
// Physical constants handed to every kernel (lattice units)
// ---------------------------------------------------------------------------
template <class C> struct Phys {
    C a, b, R, cv, mu, eta, k, kappa;
    C inv_cv, k_over_mu, eta_over_mu;
    C sgn_eps;  // dead zone of the upwind switch
};

// van der Waals pressure (eq. Pvdw)
template <class C> __device__ __forceinline__ C vdw_pressure(const Phys<C> &p, C rho, C T) {
    return rho * p.R * T / (C(1) - p.b * rho) - p.a * rho * rho;
}
// adiabatic sound speed squared (eq. vdW_speed_of_sound)
template <class C> __device__ __forceinline__ C vdw_cs2(const Phys<C> &p, C rho, C T) {
    C omb = C(1) - p.b * rho;
    return p.R * T * (C(1) + p.R * p.inv_cv) / (omb * omb) - C(2) * p.a * rho;
}

// ---------------------------------------------------------------------------
// Boundary index rules for an offset of at most one cell
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap1(int v, int n, int clamp) {
    if (v < 0) return clamp ? 0 : v + n;
    if (v >= n) return clamp ? n - 1 : v - n;
    return v;
}

struct Grid {
    int nx, ny, nz;
    int clampx, clampy, clampz;
    long long N;
};

// Internal population layout, plane-major: pops[(z Q + i) nx ny + y nx + x].
// The Q populations of one plane lie within Q nx ny values, so a kernel
// addresses a plane with one 64-bit base and 32-bit offsets.  (The public
// layout of lbm_get/set_populations stays pops[i N + cell].)
template <int Q> __host__ __device__ __forceinline__ long long pop_index(const Grid &g, int i, long long z, long long xy) {
    return (z * Q + i) * ((long long)g.nx * g.ny) + xy;
}

// ---------------------------------------------------------------------------
// Population storage forms.  load() returns the population in the compute
// type; enc() encodes it; dev() returns its deviation from the per-direction
// reference (exact for the 16-bit forms, which store the deviation rounded to
// nearest even; one subtraction for the wide forms, exact while the value is
// within a factor two of the reference).  Moment sums over deviations keep
// the large, nearly constant part out of the rounding.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN -> quiet NaN
    uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7fffu + lsb) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ uint16_t f32_to_f16_rne(float v) {
    _Float16 h = (_Float16)v;  // hardware conversion, round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

struct StoreF64 {
    using T = double;
    using C = double;
    static constexpr int bytes = 8;
    __device__ static __forceinline__ C load(const T *p, long long j, C) { return p[j]; }
    __device__ static __forceinline__ T enc(C v, C) { return v; }
    __device__ static __forceinline__ C dev(const T *p, long long j, C ref) { return p[j] - ref; }
};
struct StoreF32 {
    using T = float;
    using C = float;
    static constexpr int bytes = 4;
    __device__ static __forceinline__ C load(const T *p, long long j, C) { return p[j]; }
    __device__ static __forceinline__ T enc(C v, C) { return v; }
    __device__ static __forceinline__ C dev(const T *p, long long j, C ref) { return p[j] - ref; }
};
struct StoreBF16 {
    using T = uint16_t;
    using C = float;
    static constexpr int bytes = 2;
    __device__ static __forceinline__ C load(const T *p, long long j, C ref) { return ref + bf16_to_f32(p[j]); }
    __device__ static __forceinline__ T enc(C v, C ref) { return f32_to_bf16_rne(v - ref); }
    __device__ static __forceinline__ C dev(const T *p, long long j, C) { return bf16_to_f32(p[j]); }
};
struct StoreF16 {
    using T = uint16_t;
    using C = float;
    static constexpr int bytes = 2;
    __device__ static __forceinline__ C load(const T *p, long long j, C ref) { return ref + f16_to_f32(p[j]); }
    __device__ static __forceinline__ T enc(C v, C ref) { return f32_to_f16_rne(v - ref); }
    __device__ static __forceinline__ C dev(const T *p, long long j, C) { return f16_to_f32(p[j]); }
};

// reference populations: storage origin of the 16-bit forms, origin of the
// moment sums for every form (zero when no reference state is given)
struct RefPops {
    float f[27];
    float g[27];
};

// ---------------------------------------------------------------------------
// Product-form factors (eq. phi) evaluated per axis.  For a velocity
// component c in {-1, 0, 1}:  Psi(0) = 1 - zeta,  Psi(+-1) = (zeta +- xi)/2.
// ---------------------------------------------------------------------------
template <class C> struct Axis3 {
    C m, z, p;  // values at c = -1, 0, +1
};
template <class C> __device__ __forceinline__ Axis3<C> psi3(C xi, C zeta) {
    Axis3<C> r;
    r.z = C(1) - zeta;
    r.p = C(0.5) * (zeta + xi);
    r.m = C(0.5) * (zeta - xi);
    return r;
}
template <class C> __device__ __forceinline__ C pick(const Axis3<C> &a, int c) {
    return c < 0 ? a.m : (c > 0 ? a.p : a.z);
}

}  // namespace lbm
