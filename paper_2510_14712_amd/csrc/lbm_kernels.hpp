// Kernels of the non-ideal DDF lattice Boltzmann step (arXiv 2510.14712,
// Section 3.2 and its flowchart).  Structure-of-arrays populations, x fastest;
// one thread per cell, grid (ceil(nx / BX), ny, nz).
//
// The stored state is the post-streaming population set at time t (what the
// flowchart initialises to the equilibria).  One step is four launches:
//   k_moments  rho, j = sum c_i f_i, G = sum g_i per cell           (eqs. def_h..)
//   k_lap      discrete Laplacian of rho                             (eq. FK)
//   k_fields   Korteweg force, u, E, T, P, h, c_s^2, Lambda per cell (eqs. FK,
//              def_u, def_E, lbm_temp, Pvdw, enthalpy, correction)
//   k_collide  gradients, shifts, attractors, relax, then stream by pushing
//              f'_i(x) to x + c_i of the other buffer
//              (eqs. fLBGK, gLBGK, LBMeq, LBMstar, LBMeqG, LBMgstar, sh_*, qc_1)
#pragma once

#include "lbm_device.hpp"

namespace lbm {

constexpr int BX = 256;

// field arrays of one step, compute precision C
template <class C> struct Fields {
    C *rho, *J, *G;      // moments (J has D components)
    C *lap;              // Laplacian of rho
    C *u, *F, *Lam;      // D components each
    C *T, *P, *h, *cs2;  // scalars
    C *sc[4];            // shock-capturing work arrays (null when off)
};

template <int D> __device__ __forceinline__ long long cell_index(const Grid &g, int x, int y, int z) {
    return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}

// neighbour of (x, y, z) shifted by s along axis a (|s| <= 1)
template <int D> __device__ __forceinline__ long long nb_axis(const Grid &g, int x, int y, int z, int a, int s) {
    if (a == 0) x = wrap1(x + s, g.nx, g.clampx);
    else if (a == 1) y = wrap1(y + s, g.ny, g.clampy);
    else z = wrap1(z + s, g.nz, g.clampz);
    return cell_index<D>(g, x, y, z);
}

// Streaming destinations along one axis of a population leaving coordinate
// v with velocity component c.  Periodic: wrap(v + c).  Zero-gradient: v + c
// when inside, and also v itself when v is the boundary cell and c points
// inward (the cell outside the wall is the boundary cell's own copy).  Returns
// the number of destinations (0, 1 or 2) written to d[].
__device__ __forceinline__ int push_axis(int v, int c, int n, int clamp, int d[2]) {
    int k = 0;
    int p = v + c;
    if (!clamp) {
        d[k++] = p < 0 ? p + n : (p >= n ? p - n : p);
        return k;
    }
    if (p >= 0 && p < n) d[k++] = p;
    if ((v == 0 && c == 1) || (v == n - 1 && c == -1)) d[k++] = v;
    return k;
}

// ---------------------------------------------------------------------------
// Equilibria from per-axis factors.  p: Psi(c; u, theta + u^2) (f^eq factors);
// q(0) = m2 - m4, q(+-1) = (m4 +- m3)/2 with the Gaussian raw moments
// m2 = theta + u^2, m3 = u^3 + 3 theta u, m4 = u^4 + 6 theta u^2 + 3 theta^2
// (the Psi weights applied to O^k(u^2) = m_{k+2} - theta m_k).  Applying the operators O_a of eq. Oa to
// E = e + |u|^2/2 and collecting the product of eq. LBMeqG gives
//   g_i = f_i (e - D theta / 2) + rho/2 sum_b q_b(c_ib) prod_{a != b} p_a(c_ia).
// ---------------------------------------------------------------------------
template <class C> struct AxisEq {
    Axis3<C> p, q;
};
template <class C> __device__ __forceinline__ AxisEq<C> axis_eq(C u, C theta) {
    AxisEq<C> r;
    C u2 = u * u;
    C m2 = theta + u2;
    C m3 = u * (u2 + C(3) * theta);
    C m4 = u2 * u2 + C(6) * theta * u2 + C(3) * theta * theta;
    r.p = psi3(u, m2);
    r.q.z = m2 - m4;
    r.q.p = C(0.5) * (m4 + m3);
    r.q.m = C(0.5) * (m4 - m3);
    return r;
}

// ---------------------------------------------------------------------------
template <int D, class S>
__global__ void __launch_bounds__(BX) k_init(Grid g, Phys<double> ph, RefPops ref, const double *__restrict__ rho,
                                             const double *__restrict__ u, const double *__restrict__ T,
                                             typename S::T *__restrict__ fo, typename S::T *__restrict__ go) {
    using C = typename S::C;
    constexpr int Q = Lattice<D>::Q;
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    long long c = cell_index<D>(g, x, y, z);
    double r = rho[c], t = T[c];
    double P, e;
    if (ph.pr) {
        const EosPoint q = pr_eos(ph, r, t);
        P = q.P;
        e = q.e;
    } else {
        P = vdw_pressure(ph, r, t);
        e = ph.cv * t - ph.a * r;
    }
    double theta = P / r;
    double eps = e - 0.5 * D * theta;
    AxisEq<double> ax[3];
    for (int a = 0; a < D; a++) ax[a] = axis_eq(u[a * g.N + c], theta);
#pragma unroll
    for (int i = 0; i < Q; i++) {
        double px = pick(ax[0].p, cx_of(i)), py = pick(ax[1].p, cy_of(i));
        double qx = pick(ax[0].q, cx_of(i)), qy = pick(ax[1].q, cy_of(i));
        double feq, gsum;
        if (D == 2) {
            feq = r * px * py;
            gsum = qx * py + px * qy;
        } else {
            double pz = pick(ax[2].p, cz_of(i)), qz = pick(ax[2].q, cz_of(i));
            feq = r * px * py * pz;
            gsum = (qx * py + px * qy) * pz + px * py * qz;
        }
        double geq = feq * eps + 0.5 * r * gsum;
        const long long pi = pop_index<Q>(g, i, z, x + (long long)g.nx * y);
        fo[pi] = S::enc((C)feq, (C)ref.f[i]);
        go[pi] = S::enc((C)geq, (C)ref.g[i]);
    }
}

// ---------------------------------------------------------------------------
template <int D, class S>
__global__ void __launch_bounds__(BX) k_moments(Grid g, RefPops ref, const typename S::T *__restrict__ fi,
                                                const typename S::T *__restrict__ gi, Fields<typename S::C> fl,
                                                int pull) {
    using C = typename S::C;
    constexpr int Q = Lattice<D>::Q;
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    long long c = cell_index<D>(g, x, y, z);
    C rho = 0, J[3] = {0, 0, 0}, G = 0;
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const long long pi = arrived_index<D>(g, i, x, y, z, pull);
        C f = S::load(fi, pi, (C)ref.f[i]);
        rho += f;
        if (cx_of(i)) J[0] += cx_of(i) > 0 ? f : -f;
        if (cy_of(i)) J[1] += cy_of(i) > 0 ? f : -f;
        if (D == 3 && cz_of(i)) J[2] += cz_of(i) > 0 ? f : -f;
        G += S::load(gi, pi, (C)ref.g[i]);
    }
    fl.rho[c] = rho;
    for (int a = 0; a < D; a++) fl.J[a * g.N + c] = J[a];
    fl.G[c] = G;
}

template <int D, class C>
__global__ void __launch_bounds__(BX) k_lap(Grid g, Fields<C> fl) {
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    long long c = cell_index<D>(g, x, y, z);
    C r0 = fl.rho[c], s = 0;
    for (int a = 0; a < D; a++)
        s += fl.rho[nb_axis<D>(g, x, y, z, a, 1)] + fl.rho[nb_axis<D>(g, x, y, z, a, -1)] - C(2) * r0;
    fl.lap[c] = s;
}

// sum over a wavefront of a per-lane count, added once per wavefront
__device__ __forceinline__ void wave_count(unsigned long long *dst, unsigned v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, (unsigned long long)v);
}

// per-cell thermodynamic fields from the moments: the exact van der Waals
// caloric inversion T = (E - u^2/2 + a rho)/c_v (eq. lbm_temp), or for
// Peng-Robinson Newton's method in FP64 from the dilute estimate (warm = 0)
// or from the cell's temperature of the previous step (warm = 1);
// newton[0] counts the iterations, newton[1] the cells (may be null)
template <int D, class C>
__global__ void __launch_bounds__(BX) k_fields(Grid g, Phys<C> ph, Fields<C> fl, int warm,
                                               unsigned long long *newton) {
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    const bool active = x < g.nx;
    if (ph.pr && newton) {
        // the wavefront's lanes all take part in the count below
        if (!active) x = g.nx - 1;
    } else if (!active) {
        return;
    }
    long long c = cell_index<D>(g, x, y, z);
    C rho = fl.rho[c];
    C inv_rho = C(1) / rho;
    C u[3], F[3], uF = 0, u2 = 0;
    for (int a = 0; a < D; a++) {
        C dl = C(0.5) * (fl.lap[nb_axis<D>(g, x, y, z, a, 1)] - fl.lap[nb_axis<D>(g, x, y, z, a, -1)]);
        F[a] = ph.kappa * rho * dl;                          // eq. FK
        u[a] = (fl.J[a * g.N + c] + C(0.5) * F[a]) * inv_rho;  // eq. def_u
        uF += u[a] * F[a];
        u2 += u[a] * u[a];
    }
    C E = (fl.G[c] + C(0.5) * uF) * inv_rho;                  // eq. def_E
    C e = E - C(0.5) * u2;
    C T, P, cs2;
    if (ph.pr) {
        int it = 0;
        const double Td = pr_temperature(ph, (double)rho, (double)e, warm ? (double)fl.T[c] : 0.0, it);
        const EosPoint q = pr_eos(ph, (double)rho, Td);
        T = (C)Td;
        P = (C)q.P;
        cs2 = (C)q.cs2;
        if (newton) {
            wave_count(&newton[0], active ? (unsigned)it : 0u);
            wave_count(&newton[1], active ? 1u : 0u);
        }
        if (!active) return;
    } else {
        T = (e + ph.a * rho) * ph.inv_cv;                      // eq. lbm_temp
        P = vdw_pressure(ph, rho, T);                          // eq. Pvdw
        cs2 = vdw_cs2(ph, rho, T);                             // eq. vdW_speed_of_sound
    }
    C theta = P * inv_rho;
    for (int a = 0; a < D; a++) {
        fl.u[a * g.N + c] = u[a];
        fl.F[a * g.N + c] = F[a];
        // Lambda_a = rho u_a^3 + 3 rho u_a (theta - 1/3)   (eq. correction)
        fl.Lam[a * g.N + c] = rho * u[a] * (u[a] * u[a] + C(3) * (theta - C(1.0 / 3.0)));
    }
    fl.T[c] = T;
    fl.P[c] = P;
    fl.h[c] = e + theta;                                       // eq. enthalpy
    fl.cs2[c] = cs2;
}

// ---------------------------------------------------------------------------
// Shock-capturing numerical transport (Section 4.4, eqs. shock_cap and
// shock_cap_k, r = 5, dx = 1), three passes over the fields of the step:
//   k_sc_grad    S = |grad u + grad u^T| / 2 and |grad s|, grad s = (c_v/T) grad T
//                - R/(rho (1 - b rho)) grad rho (eq. ds_vdW), central differences
//   k_sc_d4      |sum_a d^4/dx_a^4| of both (central fourth differences)
//   k_sc_filter  the truncated Gaussian filter along one axis (launched per axis)
// k_collide then adds rho C_mu fS, rho C_eta fS and rho c_s C_k fs to mu, eta,
// k of the cell.  Indices beyond a zero-gradient wall clamp, periodic ones wrap.
__device__ __forceinline__ int wrap_any(int v, int n, int clamp) {
    if (clamp) return v < 0 ? 0 : (v >= n ? n - 1 : v);
    v %= n;
    return v < 0 ? v + n : v;
}
template <int D> __device__ __forceinline__ long long nb_axis_n(const Grid &g, int x, int y, int z, int a, int s) {
    if (a == 0) x = wrap_any(x + s, g.nx, g.clampx);
    else if (a == 1) y = wrap_any(y + s, g.ny, g.clampy);
    else z = wrap_any(z + s, g.nz, g.clampz);
    return cell_index<D>(g, x, y, z);
}

constexpr int SC_RADIUS = 4;  // filter taps -4 .. 4
template <class C> struct ScFilter {
    C w[2 * SC_RADIUS + 1];
};

template <int D, class C>
__global__ void __launch_bounds__(BX) k_sc_grad(Grid g, Phys<C> ph, Fields<C> fl) {
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const long long N = g.N, c = cell_index<D>(g, x, y, z);
    C G[3][3];  // G[a][b] = d u_a / d x_b
    const C rho = fl.rho[c], T = fl.T[c];
    // ds = (c_v / T) dT - (dP/dT)_rho / rho^2 drho; van der Waals: the second
    // coefficient is R / (rho (1 - b rho))
    C cT, cr;
    if (ph.pr) {
        const EosPoint q = pr_eos(ph, (double)rho, (double)T);
        cT = (C)(q.cv / (double)T);
        cr = (C)(q.dPdT / ((double)rho * (double)rho));
    }
    C g2 = 0;
    for (int b = 0; b < D; b++) {
        const long long cp = nb_axis<D>(g, x, y, z, b, 1), cm = nb_axis<D>(g, x, y, z, b, -1);
        for (int a = 0; a < D; a++) G[a][b] = C(0.5) * (fl.u[a * N + cp] - fl.u[a * N + cm]);
        const C dT = C(0.5) * (fl.T[cp] - fl.T[cm]), dr = C(0.5) * (fl.rho[cp] - fl.rho[cm]);
        const C ds = ph.pr ? cT * dT - cr * dr : ph.cv / T * dT - ph.R / (rho * (C(1) - ph.b * rho)) * dr;
        g2 += ds * ds;
    }
    C ss = 0;
    for (int a = 0; a < D; a++)
        for (int b = 0; b < D; b++) ss += (G[a][b] + G[b][a]) * (G[a][b] + G[b][a]);
    fl.sc[0][c] = C(0.5) * sqrt(ss);
    fl.sc[1][c] = sqrt(g2);
}

template <int D, class C>
__global__ void __launch_bounds__(BX) k_sc_d4(Grid g, const C *__restrict__ a_in, const C *__restrict__ b_in,
                                              C *__restrict__ a_out, C *__restrict__ b_out) {
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const long long c = cell_index<D>(g, x, y, z);
    C sa = 0, sb = 0;
    for (int a = 0; a < D; a++) {
        const long long p1 = nb_axis_n<D>(g, x, y, z, a, 1), p2 = nb_axis_n<D>(g, x, y, z, a, 2);
        const long long m1 = nb_axis_n<D>(g, x, y, z, a, -1), m2 = nb_axis_n<D>(g, x, y, z, a, -2);
        sa += a_in[p2] - C(4) * a_in[p1] + C(6) * a_in[c] - C(4) * a_in[m1] + a_in[m2];
        sb += b_in[p2] - C(4) * b_in[p1] + C(6) * b_in[c] - C(4) * b_in[m1] + b_in[m2];
    }
    a_out[c] = fabs(sa);
    b_out[c] = fabs(sb);
}

template <int D, class C>
__global__ void __launch_bounds__(BX) k_sc_filter(Grid g, int axis, ScFilter<C> f, const C *__restrict__ a_in,
                                                  const C *__restrict__ b_in, C *__restrict__ a_out,
                                                  C *__restrict__ b_out) {
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const long long c = cell_index<D>(g, x, y, z);
    C sa = 0, sb = 0;
    for (int j = -SC_RADIUS; j <= SC_RADIUS; j++) {
        const long long n = nb_axis_n<D>(g, x, y, z, axis, j);
        sa += f.w[j + SC_RADIUS] * a_in[n];
        sb += f.w[j + SC_RADIUS] * b_in[n];
    }
    a_out[c] = sa;
    b_out[c] = sb;
}

// ---------------------------------------------------------------------------
// Diffuse-reflection walls at x = -1 and x = nx (the thermal Couette flow of
// Section 4.1; the paper does not state its wall treatment).  Each ghost cell
// beyond a wall absorbs the populations leaving the domain into it and
// re-emits equilibria of the wall state -- u_w, T_w, and the thermodynamics of
// the boundary cell next to it (theta_w = P(rho_b, T_w)/rho_b, e_w = e(rho_b,
// T_w)) -- scaled to the absorbed mass, so no mass crosses the wall.  The
// central differences of u, T, h and Lambda at a boundary cell take the
// ghost's values; rho, its Laplacian and the shock-capturing stencils stay
// zero-gradient.  k_collide writes the leaving post-collision populations to
// the ghost buffer gb[side][(z ny + y) Q + i]; k_wall_emit then writes what
// each ghost emits.
template <class C> struct WallGhost {
    C u[3], T, theta, e, h;
};
template <class C> __device__ __forceinline__ WallGhost<C> wall_ghost(const Phys<C> &ph, const Walls &w, int side,
                                                                      C rho_b) {
    WallGhost<C> gs;
    for (int a = 0; a < 3; a++) gs.u[a] = (C)w.u[side][a];
    gs.T = (C)w.T[side];
    C P, e;
    if (ph.pr) {
        const EosPoint q = pr_eos(ph, (double)rho_b, (double)gs.T);
        P = (C)q.P;
        e = (C)q.e;
    } else {
        P = vdw_pressure(ph, rho_b, gs.T);
        e = ph.cv * gs.T - ph.a * rho_b;
    }
    gs.theta = P / rho_b;
    gs.e = e;
    gs.h = e + gs.theta;
    return gs;
}

template <int D, class S>
__global__ void __launch_bounds__(64) k_wall_emit(Grid g, Phys<typename S::C> ph, RefPops ref, Walls w,
                                                  Fields<typename S::C> fl, const typename S::C *__restrict__ gb,
                                                  typename S::T *__restrict__ fo, typename S::T *__restrict__ go) {
    using C = typename S::C;
    constexpr int Q = Lattice<D>::Q;
    const int yg = blockIdx.x * 64 + threadIdx.x, zg = blockIdx.y, side = blockIdx.z;
    if (yg >= g.ny) return;
    const int xb = side ? g.nx - 1 : 0;
    const int cin = side ? -1 : 1;  // x component of the emitted directions
    const C rho_b = fl.rho[cell_index<D>(g, xb, yg, zg)];
    const WallGhost<C> gs = wall_ghost(ph, w, side, rho_b);
    const C *src = gb + ((size_t)side * g.ny * g.nz + (size_t)zg * g.ny + yg) * Q;
    C m = 0;
    for (int j = 0; j < Q; j++)
        if (cx_of(j) == -cin) m += src[j];
    AxisEq<C> ax[3];
    for (int a = 0; a < D; a++) ax[a] = axis_eq(gs.u[a], gs.theta);
    auto pz_of = [&](int i) { return D == 3 ? pick(ax[2].p, cz_of(i)) : C(1); };
    C sm = 0;
    for (int j = 0; j < Q; j++)
        if (cx_of(j) == cin) sm += pick(ax[0].p, cx_of(j)) * pick(ax[1].p, cy_of(j)) * pz_of(j);
    const C rg = m / sm;
    const C eps = gs.e - C(0.5 * D) * gs.theta;
    for (int i = 0; i < Q; i++) {
        if (cx_of(i) != cin) continue;
        const C px = pick(ax[0].p, cx_of(i)), py = pick(ax[1].p, cy_of(i));
        const C qx = pick(ax[0].q, cx_of(i)), qy = pick(ax[1].q, cy_of(i));
        C feq, gsum;
        if (D == 2) {
            feq = rg * px * py;
            gsum = qx * py + px * qy;
        } else {
            const C pz = pick(ax[2].p, cz_of(i)), qz = pick(ax[2].q, cz_of(i));
            feq = rg * px * py * pz;
            gsum = (qx * py + px * qy) * pz + px * py * qz;
        }
        const C geq = feq * eps + C(0.5) * rg * gsum;
        const int yd = wrap1(yg + cy_of(i), g.ny, 0), zd = D == 3 ? wrap1(zg + cz_of(i), g.nz, 0) : 0;
        const long long d = pop_index<Q>(g, i, zd, xb + (long long)g.nx * yd);
        fo[d] = S::enc(feq, (C)ref.f[i]);
        go[d] = S::enc(geq, (C)ref.g[i]);
    }
}

// ---------------------------------------------------------------------------
// fS, fs: filtered |grad^4 S| and |grad^4 |grad s|| of the shock-capturing
// passes, or null without shock capturing; w, gb: wall states and ghost
// buffer (used when g.wallx)
template <int D, class S>
__global__ void __launch_bounds__(BX) k_collide(Grid g, Phys<typename S::C> ph, RefPops ref,
                                                const typename S::T *__restrict__ fi,
                                                const typename S::T *__restrict__ gi, Fields<typename S::C> fl,
                                                typename S::T *__restrict__ fo, typename S::T *__restrict__ go,
                                                const typename S::C *__restrict__ fS,
                                                const typename S::C *__restrict__ fs, Walls w,
                                                typename S::C *__restrict__ gb) {
    using C = typename S::C;
    constexpr int Q = Lattice<D>::Q;
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const long long N = g.N;
    long long c = cell_index<D>(g, x, y, z);
    C rho = fl.rho[c], P = fl.P[c], T = fl.T[c];
    // transport coefficients of the cell: the constants plus the numerical
    // contributions of the shock-capturing scheme (Section 4.4)
    C mu = ph.mu, eta_over_mu = ph.eta_over_mu, k_over_mu = ph.k_over_mu;
    if (fS) {
        const C cs = sqrt(fl.cs2[c] > C(0) ? fl.cs2[c] : C(0));
        mu = ph.mu + rho * ph.sc_cmu * fS[c];
        const C eta = ph.eta + rho * ph.sc_ceta * fS[c];
        const C kk = ph.k + rho * cs * ph.sc_ck * fs[c];
        eta_over_mu = eta / mu;
        k_over_mu = kk / mu;
    }
    C inv_rho = C(1) / rho;
    C theta = P * inv_rho;
    C u[3], F[3], divu = 0, qc[3], Phi[3], FF = 0;
    for (int a = 0; a < D; a++) {
        long long cp = nb_axis<D>(g, x, y, z, a, 1), cm = nb_axis<D>(g, x, y, z, a, -1);
        u[a] = fl.u[a * N + c];
        F[a] = fl.F[a * N + c];
        FF += F[a] * F[a];
        // u_a, h, T, Lambda_a at x - e_a ([0]) and x + e_a ([1]): the
        // neighbours', or a wall ghost's
        C nu[2] = {fl.u[a * N + cm], fl.u[a * N + cp]}, nh[2] = {fl.h[cm], fl.h[cp]};
        C nT[2] = {fl.T[cm], fl.T[cp]}, nL[2] = {fl.Lam[a * N + cm], fl.Lam[a * N + cp]};
        if (a == 0 && g.wallx) {
            for (int k = 0; k < 2; k++) {
                if (!(k == 0 ? x == 0 : x == g.nx - 1)) continue;
                const WallGhost<C> gs = wall_ghost(ph, w, k, rho);
                nu[k] = gs.u[0];
                nh[k] = gs.h;
                nT[k] = gs.T;
                nL[k] = rho * gs.u[0] * gs.u[0] * gs.u[0] + C(3) * rho * gs.u[0] * (gs.theta - C(1.0 / 3.0));
            }
        }
        divu += C(0.5) * (nu[1] - nu[0]);
        C dh = C(0.5) * (nh[1] - nh[0]);
        C dT = C(0.5) * (nT[1] - nT[0]);
        qc[a] = P * (dh - k_over_mu * dT);                     // eq. qc_1
        // upwind-biased d_a Lambda_a by sgn(u_a); |u_a| <= eps gives the average
        C L0 = fl.Lam[a * N + c];
        C dL;
        if (u[a] > ph.sgn_eps) dL = L0 - nL[0];
        else if (u[a] < -ph.sgn_eps) dL = nL[1] - L0;
        else dL = C(0.5) * (nL[1] - nL[0]);
        Phi[a] = -dL * inv_rho;                                // eq. correction
    }
    C beta = P / (P + C(2) * mu);                              // eq. beta_main with tau = mu / P
    C alpha = C(D + 2) / C(D) - rho * fl.cs2[c] / P - eta_over_mu;  // eq. corr_bulk
    C thetas = theta + alpha * theta * divu;                   // eq. sh_temp_1
    C e, es;
    if (ph.pr) {
        // e(rho, T) by the caloric relation; e(rho, T*) as the energy the
        // shift of eq. sh_T_1 stands for, e - |F|^2 / (2 rho^2) (exact for an
        // energy linear in T, and keeps the collision's energy change u . F)
        e = (C)pr_eos(ph, (double)rho, (double)T).e;
        es = e - FF * inv_rho * inv_rho * C(0.5);
    } else {
        C Ts = T - FF * inv_rho * inv_rho * C(0.5) * ph.inv_cv;  // eq. sh_T_1
        e = ph.cv * T - ph.a * rho;                            // e(rho, T), eq. de_vdW
        es = ph.cv * Ts - ph.a * rho;                          // e(rho, T*)
    }
    C eps_eq = e - C(0.5 * D) * theta;
    C eps_st = es - C(0.5 * D) * thetas;

    AxisEq<C> eq[3], st[3];
    Axis3<C> pf[3];
    for (int a = 0; a < D; a++) {
        C us = u[a] + F[a] * inv_rho;                          // eq. sh_vel_1
        eq[a] = axis_eq(u[a], theta);
        st[a] = axis_eq(us, thetas);
        pf[a] = psi3(us, thetas + us * us + Phi[a]);           // eq. zetastar
    }
    C w_keep = C(1) - C(2) * beta, w_eq = C(3) * beta - C(1), w_st = C(1) - beta;
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const int ix = cx_of(i), iy = cy_of(i), iz = D == 3 ? cz_of(i) : 0;
        C px = pick(eq[0].p, ix), py = pick(eq[1].p, iy);
        C qx = pick(eq[0].q, ix), qy = pick(eq[1].q, iy);
        C sx = pick(st[0].p, ix), sy = pick(st[1].p, iy);
        C tx = pick(st[0].q, ix), ty = pick(st[1].q, iy);
        C fsx = pick(pf[0], ix), fsy = pick(pf[1], iy);
        C feq, geqs, fst, gsts;
        if (D == 2) {
            feq = rho * px * py;
            geqs = qx * py + px * qy;
            fst = rho * fsx * fsy;
            gsts = tx * sy + sx * ty;
        } else {
            C pz = pick(eq[2].p, iz), qz = pick(eq[2].q, iz);
            C sz = pick(st[2].p, iz), tz = pick(st[2].q, iz);
            C fsz = pick(pf[2], iz);
            feq = rho * px * py * pz;
            geqs = (qx * py + px * qy) * pz + px * py * qz;
            fst = rho * fsx * fsy * fsz;
            gsts = (tx * sy + sx * ty) * sz + sx * sy * tz;
        }
        C geq = feq * eps_eq + C(0.5) * rho * geqs;
        C gst = rho * (sx * sy * (D == 3 ? pick(st[2].p, iz) : C(1))) * eps_st + C(0.5) * rho * gsts;
        if (csq_of<D>(i) == 1) {                               // eq. LBMgstar
            C cq = ix ? (ix > 0 ? qc[0] : -qc[0]) : (iy ? (iy > 0 ? qc[1] : -qc[1]) : (iz > 0 ? qc[2] : -qc[2]));
            gst += C(0.5) * cq;
        }
        const long long pi = pop_index<Q>(g, i, z, x + (long long)g.nx * y);
        C f = S::load(fi, pi, (C)ref.f[i]);
        C gg = S::load(gi, pi, (C)ref.g[i]);
        // eqs. fLBGK, gLBGK: f + 2 beta (f^eq - f) + (1 - beta)(f* - f^eq)
        C fn = w_keep * f + w_eq * feq + w_st * fst;
        C gn = w_keep * gg + w_eq * geq + w_st * gst;
        typename S::T fe = S::enc(fn, (C)ref.f[i]), ge = S::enc(gn, (C)ref.g[i]);
        int dx[2], dy[2], dz[2] = {0, 0};
        int nxd;
        if (g.wallx) {
            // walls: a population leaving through one goes to its ghost
            const int xd = x + ix;
            nxd = (xd >= 0 && xd < g.nx) ? 1 : 0;
            dx[0] = xd;
            if (!nxd) {
                const int yg = wrap1(y + iy, g.ny, 0), zg = D == 3 ? wrap1(z + iz, g.nz, 0) : 0;
                gb[((size_t)(xd < 0 ? 0 : 1) * g.ny * g.nz + (size_t)zg * g.ny + yg) * Q + i] = fn;
            }
        } else {
            nxd = push_axis(x, ix, g.nx, g.clampx, dx);
        }
        int nyd = push_axis(y, iy, g.ny, g.clampy, dy);
        int nzd = D == 3 ? push_axis(z, iz, g.nz, g.clampz, dz) : 1;
        for (int a = 0; a < nxd; a++)
            for (int b = 0; b < nyd; b++)
                for (int cc = 0; cc < nzd; cc++) {
                    const long long d = pop_index<Q>(g, i, dz[cc], dx[a] + (long long)g.nx * dy[b]);
                    fo[d] = fe;
                    go[d] = ge;
                }
    }
}

}  // namespace lbm
