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
    C sc_cmu, sc_ceta, sc_ck;  // shock-capturing coefficients (zero: off)
    int pr;                    // 1: Peng-Robinson (a, b, R and the fields below); 0: van der Waals
    double pr_m, pr_Tc, pr_c0, pr_c1;
};

// ---------------------------------------------------------------------------
// Peng-Robinson equation of state (the paper's example of a fluid whose
// temperature needs a node-wise non-linear solve, Section 3.2 after eq.
// lbm_temp), in FP64:
//   P = rho R T / (1 - b rho) - a alpha(T) rho^2 / (1 + 2 b rho - b^2 rho^2),
//   alpha = (1 + m (1 - s))^2, s = sqrt(T / Tc),
//   e = c0 T + c1 T^2 / 2 - a (1 + m)(1 + m (1 - s)) L(rho)   (c_v0 = c0 + c1 T),
//   L = ln[(1 + (1 + sqrt2) b rho) / (1 + (1 - sqrt2) b rho)] / (2 sqrt2 b),
// the energy departure being the integral of (P - T dP/dT)/rho^2 over
// density; c_v = c_v0 + a T alpha'' L; c_s^2 = (dP/drho)_T + T (dP/dT)^2 /
// (rho^2 c_v) (eq. speed_of_sound).
// ---------------------------------------------------------------------------
struct EosPoint {
    double P, e, cv, cs2, dPdT;
};
template <class C> __device__ __forceinline__ EosPoint pr_eos(const Phys<C> &ph, double rho, double T) {
    const double a = (double)ph.a, b = (double)ph.b, R = (double)ph.R, m = ph.pr_m;
    const double sq = sqrt(T * ph.pr_Tc);
    const double k = 1.0 + m * (1.0 - sqrt(T / ph.pr_Tc));
    const double alpha = k * k;
    const double dalpha = -m * k / sq;
    const double d2alpha = 0.5 * m * (1.0 + m) / (T * sq);
    const double den = 1.0 + 2.0 * b * rho - b * b * rho * rho;
    const double omb = 1.0 - b * rho;
    const double r2 = 1.4142135623730951;
    const double L = log((1.0 + (1.0 + r2) * b * rho) / (1.0 + (1.0 - r2) * b * rho)) / (2.0 * r2 * b);
    EosPoint o;
    o.P = rho * R * T / omb - a * alpha * rho * rho / den;
    o.e = ph.pr_c0 * T + 0.5 * ph.pr_c1 * T * T - a * (1.0 + m) * k * L;
    o.cv = ph.pr_c0 + ph.pr_c1 * T + a * T * d2alpha * L;
    o.dPdT = rho * R / omb - a * dalpha * rho * rho / den;
    const double dPdrho = R * T / (omb * omb) - a * alpha * (2.0 * rho * den - rho * rho * (2.0 * b - 2.0 * b * b * rho)) /
                                                    (den * den);
    o.cs2 = dPdrho + T * o.dPdT * o.dPdT / (rho * rho * o.cv);
    return o;
}
// Newton's method on e(rho, T) = e from T0 (a non-positive or non-finite
// start is replaced by the dilute estimate e / c0, else T_c), a step that
// would leave T > 0 halved; converged when the step is below 1e-15 T.
// `iters` receives the iterations taken (50 at most).
template <class C>
__device__ __forceinline__ double pr_temperature(const Phys<C> &ph, double rho, double e, double T0, int &iters) {
    double t = T0;
    if (!(t > 1e-3 * ph.pr_Tc)) t = e / ph.pr_c0;
    if (!(t > 1e-3 * ph.pr_Tc)) t = ph.pr_Tc;
    iters = 0;
    for (int it = 1; it <= 50; it++) {
        const EosPoint q = pr_eos(ph, rho, t);
        double dt = (q.e - e) / q.cv;
        double tn = t - dt;
        while (!(tn > 0.0) && fabs(dt) > 1e-300) {
            dt *= 0.5;
            tn = t - dt;
        }
        t = tn;
        iters = it;
        if (!(fabs(dt) > 1e-15 * t)) break;
    }
    return t;
}

// van der Waals pressure (eq. Pvdw)
template <class C> __device__ __forceinline__ C vdw_pressure(const Phys<C> &p, C rho, C T) {
    return rho * p.R * T / (C(1) - p.b * rho) - p.a * rho * rho;
}
// adiabatic sound speed squared (eq. vdW_speed_of_sound)
template <class C> __device__ __forceinline__ C vdw_cs2(const Phys<C> &p, C rho, C T) {
    C omb = C(1) - p.b * rho;
    return p.R * T * (C(1) + p.R * p.inv_cv) / (omb * omb) - C(2) * p.a * rho;
}

// a / b in the form's arithmetic: exact in FP64; in FP32 a times the hardware
// reciprocal (1 ulp), a tenth of the instructions of the correctly rounded
// division, well inside the FP32 form's error against the FP64 method
template <class C> __device__ __forceinline__ C fdiv(C a, C b) { return a / b; }
template <> __device__ __forceinline__ float fdiv<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// pressure and adiabatic sound speed squared together (eqs. Pvdw,
// vdW_speed_of_sound); FP32 shares one reciprocal of 1 - b rho, FP64 takes the
// two closed forms as written
template <class C> __device__ __forceinline__ void vdw_p_cs2(const Phys<C> &p, C rho, C T, C &P, C &cs2) {
    P = vdw_pressure(p, rho, T);
    cs2 = vdw_cs2(p, rho, T);
}
template <> __device__ __forceinline__ void vdw_p_cs2<float>(const Phys<float> &p, float rho, float T, float &P,
                                                             float &cs2) {
    const float r = __builtin_amdgcn_rcpf(1.0f - p.b * rho);
    P = rho * p.R * T * r - p.a * rho * rho;
    cs2 = p.R * T * (1.0f + p.R * p.inv_cv) * (r * r) - 2.0f * p.a * rho;
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
    int wallx;  // 1: diffuse-reflection walls at x = -1 and x = nx (clampx is then 1 too)
};

// wall states of the x walls: [0] at x = -1, [1] at x = nx
struct Walls {
    double u[2][3];
    double T[2];
};

// Internal population layout: plane-major, with f_i and g_i of a cell side by
// side, pops[((z Q + i) nx ny + y nx + x) 2 + {0: f, 1: g}].  The Q population
// pairs of one plane lie within 2 Q nx ny values, so a kernel addresses a
// plane with one 64-bit base and 32-bit offsets, and one load or store moves
// both populations of a direction.  pop_index gives the element index of f;
// the g array is the same buffer offset by one element, so f[j] and g[j]
// address the pair.  (The public layout of lbm_get/set_populations stays
// pops[i N + cell].)
template <int Q> __host__ __device__ __forceinline__ long long pop_index(const Grid &g, int i, long long z, long long xy) {
    return 2 * ((z * Q + i) * ((long long)g.nx * g.ny) + xy);
}

// Stored population sets come in two forms.  After initialisation (and after
// lbm_set_populations) the set holds the arrived populations f_i(x) that the
// next collision uses in place.  The fused step stores the post-collision set
// instead and streams on the way in: the population arriving at x with
// velocity c_i is read from x - c_i (wrapped on a periodic axis, clamped to
// the edge cell on a zero-gradient axis, which is the streaming rule of
// Sec. 3.2 with the boundary reading of the oracle).  `pull` selects the
// form: 0 reads x itself, 1 reads x - c.
__host__ __device__ __forceinline__ int pull_coord(int x, int c, int n, int clamp, int pull) {
    const int p = x - pull * c;
    if (clamp) return p < 0 ? 0 : (p >= n ? n - 1 : p);
    return p < 0 ? p + n : (p >= n ? p - n : p);
}
// index of arrived population i of cell (x, y, z) in a stored set of either
// form
template <int D>
__host__ __device__ __forceinline__ long long arrived_index(const Grid &g, int i, int x, int y, int z, int pull) {
    constexpr int Q = D == 2 ? 9 : 27;
    const int sx = pull_coord(x, cx_of(i), g.nx, g.clampx, pull);
    const int sy = pull_coord(y, cy_of(i), g.ny, g.clampy, pull);
    const int sz = D == 3 ? pull_coord(z, cz_of(i), g.nz, g.clampz, pull) : 0;
    return pop_index<Q>(g, i, sz, sx + (long long)g.nx * sy);
}

// ---------------------------------------------------------------------------
// Population storage forms.  load() returns the population in the compute
// type; enc() encodes it; dev() returns its deviation from the per-direction
// reference (exact for the 16-bit forms, which store the deviation rounded to
// nearest even; one subtraction for the wide forms, exact while the value is
// within a factor two of the reference).  Moment sums over deviations keep
// the large, nearly constant part out of the rounding.
// ---------------------------------------------------------------------------
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
// round to nearest, ties to even, by the hardware convert (v_cvt_pk_bf16_f32);
// a NaN gives a quiet NaN whose payload is not specified
__device__ __forceinline__ uint16_t bf16_hw(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
// two values in one convert: a in the low half, b in the high half
__device__ __forceinline__ uint32_t bf16x2_hw(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
}
// the codec's definition: as bf16_hw, every NaN to the quiet NaN 0x7fc0
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v) { return v != v ? (uint16_t)0x7fc0 : bf16_hw(v); }
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ uint16_t f32_to_f16_rne(float v) {
    _Float16 h = (_Float16)v;  // hardware conversion, round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

struct StoreF64 {
    using T = double;
    using C = double;
    using X = double;  // exchange type (deviation as computed)
    static constexpr int bytes = 8;
    __device__ static __forceinline__ X xenc(C d) { return d; }
    __device__ static __forceinline__ C xdec(X x) { return x; }
    __device__ static __forceinline__ C load(const T *p, long long j, C) { return p[j]; }
    __device__ static __forceinline__ T enc(C v, C) { return v; }
    __device__ static __forceinline__ void enc2(C a, C ra, C b, C rb, T &ea, T &eb) {
        ea = enc(a, ra);
        eb = enc(b, rb);
    }
    __device__ static __forceinline__ C dev(const T *p, long long j, C ref) { return p[j] - ref; }
};
struct StoreF32 {
    using T = float;
    using C = float;
    using X = float;
    static constexpr int bytes = 4;
    __device__ static __forceinline__ X xenc(C d) { return d; }
    __device__ static __forceinline__ C xdec(X x) { return x; }
    __device__ static __forceinline__ C load(const T *p, long long j, C) { return p[j]; }
    __device__ static __forceinline__ T enc(C v, C) { return v; }
    __device__ static __forceinline__ void enc2(C a, C ra, C b, C rb, T &ea, T &eb) {
        ea = enc(a, ra);
        eb = enc(b, rb);
    }
    __device__ static __forceinline__ C dev(const T *p, long long j, C ref) { return p[j] - ref; }
};
struct StoreBF16 {
    using T = uint16_t;
    using C = float;
    using X = uint16_t;  // a stored deviation is a BF16 value: its code, exactly
    static constexpr int bytes = 2;
    __device__ static __forceinline__ X xenc(C d) { return (X)(__float_as_uint(d) >> 16); }
    __device__ static __forceinline__ C xdec(X x) { return bf16_to_f32(x); }
    __device__ static __forceinline__ C load(const T *p, long long j, C ref) { return ref + bf16_to_f32(p[j]); }
    __device__ static __forceinline__ T enc(C v, C ref) { return bf16_hw(v - ref); }
    __device__ static __forceinline__ C dev(const T *p, long long j, C) { return bf16_to_f32(p[j]); }
    // one convert per population: the same bits as converting the pair in one
    // v_cvt_pk_bf16_f32, which held more registers through the fused step's
    // store loop (253 against 244 VGPRs, and a spill in the 16-bit instance
    // that completes its input moments)
    __device__ static __forceinline__ void enc2(C a, C ra, C b, C rb, T &ea, T &eb) {
        ea = enc(a, ra);
        eb = enc(b, rb);
    }
};
struct StoreF16 {
    using T = uint16_t;
    using C = float;
    using X = uint16_t;  // an FP16 value: its code, exactly
    static constexpr int bytes = 2;
    __device__ static __forceinline__ X xenc(C d) { return f32_to_f16_rne(d); }
    __device__ static __forceinline__ C xdec(X x) { return f16_to_f32(x); }
    __device__ static __forceinline__ C load(const T *p, long long j, C ref) { return ref + f16_to_f32(p[j]); }
    __device__ static __forceinline__ T enc(C v, C ref) { return f32_to_f16_rne(v - ref); }
    __device__ static __forceinline__ void enc2(C a, C ra, C b, C rb, T &ea, T &eb) {
        ea = enc(a, ra);
        eb = enc(b, rb);
    }
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
