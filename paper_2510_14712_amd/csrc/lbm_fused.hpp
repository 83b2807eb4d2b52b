// Single-pass fused step: every population is read once and written once per
// step (Section 3.2 and its flowchart: moments -> Korteweg force -> u, E, T,
// P, Phi, q^c -> attractors -> collide and stream).
//
// Decomposition.  A workgroup owns a TX x TY tile of (x, y) columns and marches
// over z.  The non-local inputs of the collision are the moments of the
// post-streaming state: rho on the L1 ball of radius 3 (Laplacian, then the
// Korteweg force at the face neighbours), j and G at the face neighbours.
// Those moments are produced by the previous step: after colliding a plane,
// the workgroup gathers the pushed populations into moment sums for every
// destination cell of the tile and of its one-cell ring (LDS, fixed order,
// one owning thread per destination).  Tile cells are written to Mc; ring
// cells are written into "inbound" slots that belong to the neighbouring tile
// (IN), one writer per slot.  A reader adds the inbound slots of a cell on a
// tile edge to Mc.  z-wrap contributions go to two extra layers of Mc / IN
// (logical planes -1 and nz) that a reader adds to planes nz-1 and 0.
//
// Per marching position z (colliding plane z):
//   rho(z+3) on R3 (tile + halo 3)  -> Laplacian L(z+2) on R2 (halo 2)
//   -> F(z+1), u, E, T, P, h, Lambda, c_s^2 on R1 (halo 1)
//   -> collide plane z (needs fields of z-1, z, z+1), push to the other buffer
//   -> moment sums of the pushed populations for planes z-1, z, z+1
//   -> plane z-1 complete: write Mc / IN.
// Ghost cells of zero-gradient axes take the field of the clamped cell.
#pragma once

#include "lbm_kernels.hpp"
#include "lbm_mlp_device.hpp"

namespace lbm {

template <int TX_, int TY_> struct Tile {
    static constexpr int TX = TX_, TY = TY_, NT = TX_ * TY_;
    static constexpr int NR = 2 * TX_ + 2 * TY_ + 4;  // inbound slots per tile, plane and field
    static constexpr int W3 = TX_ + 6, H3 = TY_ + 6, R3 = W3 * H3;
    static constexpr int W2 = TX_ + 4, H2 = TY_ + 4, R2 = W2 * H2;
    static constexpr int W1 = TX_ + 2, H1 = TY_ + 2, R1 = W1 * H1;
    // inbound slot offsets
    static constexpr int FROM_L = 0, FROM_R = TY_, FROM_B = 2 * TY_, FROM_T = 2 * TY_ + TX_;
    static constexpr int FROM_BL = 2 * TY_ + 2 * TX_, FROM_BR = FROM_BL + 1, FROM_TL = FROM_BL + 2,
                         FROM_TR = FROM_BL + 3;
};

template <class C, class T> struct FusedArgs {
    Grid g;
    Phys<C> ph;
    RefPops ref;
    int ntx, nty, nlayer;  // tiles along x, y; moment layers (nz + 2 for D = 3, 1 for D = 2)
    const T *fi, *gi;
    T *fo, *go;
    const C *Mci, *INi;
    C *Mco, *INo;
    // surrogate equation of state (used when the kernel is built with MLP)
    const float *mlpP;        // FP32 parameters
    const uint16_t *mlpW2b;   // BF16 copy of the hidden weights
    const float *mlpNorm;     // normalisation constants
    float mlpTol;             // residual threshold
    unsigned long long *mlpCount;  // [0] fallbacks, [1] evaluations
};

// layer of logical plane p (-1 .. nz) in the moment arrays
template <int D> __device__ __forceinline__ int layer_of(int p) { return D == 3 ? p + 1 : 0; }

// Moment k of the post-streaming state at global (gx, gy) of physical plane
// z: own-tile value plus inbound contributions, plus the z-wrap layers.
template <int D, class TL, class C, class T>
__device__ __forceinline__ C moment_at(const FusedArgs<C, T> &a, int gx, int gy, int z, int k) {
    const Grid &g = a.g;
    const int tx = gx / TL::TX, ty = gy / TL::TY;
    const int lx = gx - tx * TL::TX, ly = gy - ty * TL::TY;
    const int w = min(TL::TX, g.nx - tx * TL::TX), h = min(TL::TY, g.ny - ty * TL::TY);
    const long long plane = (long long)g.nx * g.ny;
    const long long tile = (long long)ty * a.ntx + tx;
    auto one = [&](int layer) -> C {
        C v = a.Mci[((long long)k * a.nlayer + layer) * plane + gx + (long long)g.nx * gy];
        const C *in = a.INi + ((tile * a.nlayer + layer) * 5 + k) * TL::NR;
        if (lx == 0) v += in[TL::FROM_L + ly];
        if (lx == w - 1) v += in[TL::FROM_R + ly];
        if (ly == 0) v += in[TL::FROM_B + lx];
        if (ly == h - 1) v += in[TL::FROM_T + lx];
        if (lx == 0 && ly == 0) v += in[TL::FROM_BL];
        if (lx == w - 1 && ly == 0) v += in[TL::FROM_BR];
        if (lx == 0 && ly == h - 1) v += in[TL::FROM_TL];
        if (lx == w - 1 && ly == h - 1) v += in[TL::FROM_TR];
        return v;
    };
    C v = one(layer_of<D>(z));
    if (D == 3) {
        if (z == g.nz - 1) v += one(layer_of<D>(-1));
        if (z == 0) v += one(layer_of<D>(g.nz));
    }
    return v;
}

// global coordinate along an axis for a tile-relative offset, and the
// effective tile-relative offset at which a field is evaluated (ghost cells of
// zero-gradient axes take the clamped cell's value)
__device__ __forceinline__ int axis_global(int t0, int rel, int n, int clamp) {
    int v = t0 + rel;
    if (clamp) return v < 0 ? 0 : (v >= n ? n - 1 : v);
    v %= n;
    return v < 0 ? v + n : v;
}
__device__ __forceinline__ int axis_eff(int t0, int rel, int n, int clamp) {
    if (!clamp) return rel;
    int v = t0 + rel;
    return v < 0 ? -t0 : (v >= n ? n - 1 - t0 : rel);
}

template <int D, class S, class TL, bool MLP>
__global__ void __launch_bounds__(TL::NT) k_fused(FusedArgs<typename S::C, typename S::T> a) {
    using C = typename S::C;
    using T = typename S::T;
    constexpr int Q = Lattice<D>::Q;
    constexpr int NZ3 = D == 3 ? 3 : 1;
    constexpr int NZ2 = D == 3 ? 2 : 1;
    constexpr int TX = TL::TX, TY = TL::TY, NT = TL::NT;
    // ring fields on R1: u_x, u_y, T, h, Lambda_x, Lambda_y
    // centre fields on tile cells: rho, u_z, F_x, F_y, F_z, P, c_s^2, Lambda_z
    enum { RUX, RUY, RT, RH, RLX, RLY, NRF };
    enum { CRHO, CUZ, CFX, CFY, CFZ, CP, CCS, CLZ, NCF };
    __shared__ C sRho[NZ3][TL::R3];
    __shared__ C sLap[NZ3][TL::R2];
    __shared__ C sRing[NZ2][NRF][TL::R1];
    __shared__ C sCen[NZ2][NCF][NT];
    __shared__ C sZm[4][NT];  // plane z-1: u_z, T, h, Lambda_z
    __shared__ C sAcc[NZ3][5][TL::R1];
    __shared__ C sX[9][NT];   // exchange of pushed populations; j, G staging before that

    const Grid &g = a.g;
    const long long N = g.N;
    const int tid = threadIdx.x;
    const int bx = blockIdx.x, by = blockIdx.y;
    const int x0 = bx * TX, y0 = by * TY;
    const int w = min(TX, g.nx - x0), h = min(TY, g.ny - y0);
    const int lx = tid % TX, ly = tid / TX;
    const bool own = lx < w && ly < h;
    const int nz = g.nz;

    auto zslot3 = [](int p) { return ((p % 3) + 3) % 3; };
    auto zslot2 = [](int p) { return p & 1; };
    auto zphys = [&](int p) { int v = p % nz; return v < 0 ? v + nz : v; };

    // rho of logical plane p on R3
    auto load_rho = [&](int p) {
        const int zp = D == 3 ? zphys(p) : 0;
        C *dst = sRho[D == 3 ? zslot3(p) : 0];
        for (int r = tid; r < TL::R3; r += NT) {
            const int i = r % TL::W3 - 3, j = r / TL::W3 - 3;
            const int gx = axis_global(x0, i, g.nx, g.clampx), gy = axis_global(y0, j, g.ny, g.clampy);
            dst[r] = moment_at<D, TL>(a, gx, gy, zp, 0);
        }
    };
    // Laplacian of logical plane p on R2
    auto make_lap = [&](int p) {
        const C *rc = sRho[D == 3 ? zslot3(p) : 0];
        const C *rm = sRho[D == 3 ? zslot3(p - 1) : 0];
        const C *rp = sRho[D == 3 ? zslot3(p + 1) : 0];
        C *dst = sLap[D == 3 ? zslot3(p) : 0];
        for (int r = tid; r < TL::R2; r += NT) {
            const int i = axis_eff(x0, r % TL::W2 - 2, g.nx, g.clampx) + 3;
            const int j = axis_eff(y0, r / TL::W2 - 2, g.ny, g.clampy) + 3;
            const int c = j * TL::W3 + i;
            C s = rc[c + 1] + rc[c - 1] - C(2) * rc[c] + rc[c + TL::W3] + rc[c - TL::W3] - C(2) * rc[c];
            if (D == 3) s += rp[c] + rm[c] - C(2) * rc[c];
            dst[r] = s;
        }
    };
    // j, G of logical plane p on R1 into the staging area (sX)
    C *sJG = &sX[0][0];  // 4 x R1 values
    static_assert(4 * TL::R1 <= 9 * NT, "staging area too small");
    auto load_jg = [&](int p) {
        const int zp = D == 3 ? zphys(p) : 0;
        for (int r = tid; r < TL::R1; r += NT) {
            const int i = r % TL::W1 - 1, j = r / TL::W1 - 1;
            const int gx = axis_global(x0, i, g.nx, g.clampx), gy = axis_global(y0, j, g.ny, g.clampy);
            for (int k = 0; k < 4; k++)
                sJG[k * TL::R1 + r] = moment_at<D, TL>(a, gx, gy, zp, 1 + k);
        }
    };
    // F, u, E, T, P, h, Lambda, c_s^2 of logical plane p on R1.  The loop is
    // uniform per wavefront (the surrogate evaluates 64 cells per wave).
    auto make_fields = [&](int p) {
        const C *lc = sLap[D == 3 ? zslot3(p) : 0];
        const C *lm = sLap[D == 3 ? zslot3(p - 1) : 0];
        const C *lp = sLap[D == 3 ? zslot3(p + 1) : 0];
        const C *rc = sRho[D == 3 ? zslot3(p) : 0];
        const int s2 = D == 3 ? zslot2(p) : 0;
        const int lane = tid & 63;
        for (int r0 = tid - lane; r0 < TL::R1; r0 += NT) {
            const bool act = r0 + lane < TL::R1;
            const int r = act ? r0 + lane : TL::R1 - 1;
            const int ri = r % TL::W1 - 1, rj = r / TL::W1 - 1;
            const int ei = axis_eff(x0, ri, g.nx, g.clampx), ej = axis_eff(y0, rj, g.ny, g.clampy);
            const int c2 = (ej + 2) * TL::W2 + ei + 2;
            const int c1 = (ej + 1) * TL::W1 + ei + 1;
            const C rho = rc[(ej + 3) * TL::W3 + ei + 3];
            const C inv_rho = C(1) / rho;
            C F[3], u[3], uF = 0, u2 = 0;
            F[0] = a.ph.kappa * rho * C(0.5) * (lc[c2 + 1] - lc[c2 - 1]);
            F[1] = a.ph.kappa * rho * C(0.5) * (lc[c2 + TL::W2] - lc[c2 - TL::W2]);
            F[2] = D == 3 ? a.ph.kappa * rho * C(0.5) * (lp[c2] - lm[c2]) : C(0);
            for (int d = 0; d < D; d++) {
                u[d] = (sJG[d * TL::R1 + c1] + C(0.5) * F[d]) * inv_rho;
                uF += u[d] * F[d];
                u2 += u[d] * u[d];
            }
            if (D == 2) u[2] = 0;
            const C E = (sJG[3 * TL::R1 + c1] + C(0.5) * uF) * inv_rho;
            const C e = E - C(0.5) * u2;
            C Tt, P, cs2;
            if constexpr (MLP) {
                // surrogate temperature, accepted when the caloric residual
                // |e(rho, T_hat) - e| / (c_v T_hat) is within the threshold;
                // otherwise one FP64 Newton step on e(rho, T) = e (exact for
                // van der Waals).  P and c_s^2 from the EOS at the accepted T.
                float x0n, x1n, yh[1];
                mlp::normalise(a.mlpNorm, (float)rho, (float)e, x0n, x1n);
                mlp::forward_wave<1>(x0n, x1n, a.mlpP, a.mlpW2b, yh);
                float Th = yh[0] * a.mlpNorm[5] + a.mlpNorm[4];
                const float res = fabsf((float)a.ph.cv * Th - (float)a.ph.a * (float)rho - (float)e) /
                                  ((float)a.ph.cv * fabsf(Th));
                const bool fb = !(res <= a.mlpTol);
                if (fb) {
                    double Td = (double)Th;
                    Td = Td - ((double)a.ph.cv * Td - (double)a.ph.a * (double)rho - (double)e) / (double)a.ph.cv;
                    Th = (float)Td;
                }
                Tt = (C)Th;
                const unsigned long long nfb = __popcll(__ballot(fb && act));
                const unsigned long long nact = __popcll(__ballot(act));
                if (lane == 0) {
                    atomicAdd(&a.mlpCount[0], nfb);
                    atomicAdd(&a.mlpCount[1], nact);
                }
            } else {
                Tt = (e + a.ph.a * rho) * a.ph.inv_cv;  // eq. lbm_temp
            }
            P = vdw_pressure(a.ph, rho, Tt);
            cs2 = vdw_cs2(a.ph, rho, Tt);
            if (!act) continue;
            const C theta = P * inv_rho;
            C Lam[3];
            for (int d = 0; d < 3; d++) Lam[d] = rho * u[d] * (u[d] * u[d] + C(3) * (theta - C(1.0 / 3.0)));
            sRing[s2][RUX][r] = u[0];
            sRing[s2][RUY][r] = u[1];
            sRing[s2][RT][r] = Tt;
            sRing[s2][RH][r] = e + theta;
            sRing[s2][RLX][r] = Lam[0];
            sRing[s2][RLY][r] = Lam[1];
            if (ri >= 0 && ri < TX && rj >= 0 && rj < TY) {
                const int t = rj * TX + ri;
                sCen[s2][CRHO][t] = rho;
                sCen[s2][CUZ][t] = u[2];
                sCen[s2][CFX][t] = F[0];
                sCen[s2][CFY][t] = F[1];
                sCen[s2][CFZ][t] = F[2];
                sCen[s2][CP][t] = P;
                sCen[s2][CCS][t] = cs2;
                sCen[s2][CLZ][t] = Lam[2];
            }
        }
    };
    // write the completed moment sums of logical plane p (tile cells to Mc,
    // ring cells to the neighbours' inbound slots), then clear the slot
    auto flush = [&](int p) {
        C *acc = &sAcc[D == 3 ? zslot3(p) : 0][0][0];
        const int layer = layer_of<D>(p);
        const int zw = D == 3 ? zphys(p) : 0;
        (void)zw;
        const long long plane = (long long)g.nx * g.ny;
        for (int r = tid; r < TL::R1; r += NT) {
            const int rx = r % TL::W1 - 1, ry = r / TL::W1 - 1;
            const bool inx = rx >= 0 && rx < w, iny = ry >= 0 && ry < h;
            if (inx && iny) {
                const long long cell = (long long)(x0 + rx) + (long long)g.nx * (y0 + ry);
                for (int k = 0; k < 5; k++) a.Mco[((long long)k * a.nlayer + layer) * plane + cell] = acc[k * TL::R1 + r];
            } else if ((rx >= -1 && rx <= w) && (ry >= -1 && ry <= h)) {
                // neighbour tile and its inbound slot
                int dx = rx < 0 ? -1 : (rx >= w ? 1 : 0);
                int dy = ry < 0 ? -1 : (ry >= h ? 1 : 0);
                int nbx = bx + dx, nby = by + dy;
                bool ok = true;
                if (nbx < 0 || nbx >= a.ntx) {
                    if (g.clampx) ok = false;
                    else nbx = (nbx + a.ntx) % a.ntx;
                }
                if (nby < 0 || nby >= a.nty) {
                    if (g.clampy) ok = false;
                    else nby = (nby + a.nty) % a.nty;
                }
                if (ok) {
                    int slot;
                    if (dy == 0) slot = dx < 0 ? TL::FROM_R + ry : TL::FROM_L + ry;
                    else if (dx == 0) slot = dy < 0 ? TL::FROM_T + rx : TL::FROM_B + rx;
                    else if (dx < 0) slot = dy < 0 ? TL::FROM_TR : TL::FROM_BR;
                    else slot = dy < 0 ? TL::FROM_TL : TL::FROM_BL;
                    const long long tile = (long long)nby * a.ntx + nbx;
                    for (int k = 0; k < 5; k++)
                        a.INo[((tile * a.nlayer + layer) * 5 + k) * TL::NR + slot] = acc[k * TL::R1 + r];
                }
            }
            for (int k = 0; k < 5; k++) acc[k * TL::R1 + r] = C(0);
        }
    };

    // -- clear the accumulators ------------------------------------------------
    for (int r = tid; r < NZ3 * 5 * TL::R1; r += NT) (&sAcc[0][0][0])[r] = C(0);

    // -- prologue --------------------------------------------------------------
    if (D == 3) {
        load_rho(-3);
        load_rho(-2);
        load_rho(-1);
        __syncthreads();
        make_lap(-2);
        __syncthreads();
        load_rho(0);
        __syncthreads();
        make_lap(-1);
        __syncthreads();
        load_rho(1);
        __syncthreads();
        make_lap(0);
        load_jg(-1);
        __syncthreads();
        make_fields(-1);
        __syncthreads();
        load_rho(2);
        __syncthreads();
        make_lap(1);
        load_jg(0);
        __syncthreads();
        make_fields(0);
        __syncthreads();
    } else {
        load_rho(0);
        load_jg(0);
        __syncthreads();
        make_lap(0);
        __syncthreads();
        make_fields(0);
        __syncthreads();
    }

    const int zend = D == 3 ? nz : 1;
    for (int z = 0; z < zend; z++) {
        // own populations of plane z (issued before the field pipeline)
        C fown[Q], gown[Q];
        const long long cell = (long long)(x0 + (own ? lx : 0)) + (long long)g.nx * ((y0 + (own ? ly : 0)) + (long long)g.ny * z);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            fown[i] = S::load(a.fi, i * N + cell, (C)a.ref.f[i]);
            gown[i] = S::load(a.gi, i * N + cell, (C)a.ref.g[i]);
        }
        if (D == 3) {
            // plane z-1's z-neighbour fields leave the two-slot ring now
            if (own) {
                const int sm = zslot2(z - 1);
                const int c1 = (ly + 1) * TL::W1 + lx + 1;
                sZm[0][tid] = sCen[sm][CUZ][tid];
                sZm[1][tid] = sRing[sm][RT][c1];
                sZm[2][tid] = sRing[sm][RH][c1];
                sZm[3][tid] = sCen[sm][CLZ][tid];
            }
            load_rho(z + 3);
            __syncthreads();
            make_lap(z + 2);
            load_jg(z + 1);
            __syncthreads();
            make_fields(z + 1);
            __syncthreads();
        }

        // -- collide the own cell of plane z ---------------------------------
        C fpost[Q], gpost[Q];
        if (own) {
            const int s0 = D == 3 ? zslot2(z) : 0, s1 = D == 3 ? zslot2(z + 1) : 0;
            const int c1 = (ly + 1) * TL::W1 + lx + 1;
            const C rho = sCen[s0][CRHO][tid], P = sCen[s0][CP][tid], Tt = sRing[s0][RT][c1];
            const C inv_rho = C(1) / rho;
            const C theta = P * inv_rho;
            C u[3] = {sRing[s0][RUX][c1], sRing[s0][RUY][c1], sCen[s0][CUZ][tid]};
            C F[3] = {sCen[s0][CFX][tid], sCen[s0][CFY][tid], sCen[s0][CFZ][tid]};
            C Lm[3], Lp[3], L0[3] = {sRing[s0][RLX][c1], sRing[s0][RLY][c1], sCen[s0][CLZ][tid]};
            C dh[3], dT[3], du = 0;
            // x, y neighbours from the R1 ring fields
            du += C(0.5) * (sRing[s0][RUX][c1 + 1] - sRing[s0][RUX][c1 - 1]);
            du += C(0.5) * (sRing[s0][RUY][c1 + TL::W1] - sRing[s0][RUY][c1 - TL::W1]);
            dh[0] = C(0.5) * (sRing[s0][RH][c1 + 1] - sRing[s0][RH][c1 - 1]);
            dh[1] = C(0.5) * (sRing[s0][RH][c1 + TL::W1] - sRing[s0][RH][c1 - TL::W1]);
            dT[0] = C(0.5) * (sRing[s0][RT][c1 + 1] - sRing[s0][RT][c1 - 1]);
            dT[1] = C(0.5) * (sRing[s0][RT][c1 + TL::W1] - sRing[s0][RT][c1 - TL::W1]);
            Lm[0] = sRing[s0][RLX][c1 - 1];
            Lp[0] = sRing[s0][RLX][c1 + 1];
            Lm[1] = sRing[s0][RLY][c1 - TL::W1];
            Lp[1] = sRing[s0][RLY][c1 + TL::W1];
            if (D == 3) {
                du += C(0.5) * (sCen[s1][CUZ][tid] - sZm[0][tid]);
                dT[2] = C(0.5) * (sRing[s1][RT][c1] - sZm[1][tid]);
                dh[2] = C(0.5) * (sRing[s1][RH][c1] - sZm[2][tid]);
                Lm[2] = sZm[3][tid];
                Lp[2] = sCen[s1][CLZ][tid];
            }
            C qc[3], Phi[3], FF = 0;
            for (int d = 0; d < D; d++) {
                FF += F[d] * F[d];
                qc[d] = P * (dh[d] - a.ph.k_over_mu * dT[d]);
                C dL;
                if (u[d] > a.ph.sgn_eps) dL = L0[d] - Lm[d];
                else if (u[d] < -a.ph.sgn_eps) dL = Lp[d] - L0[d];
                else dL = C(0.5) * (Lp[d] - Lm[d]);
                Phi[d] = -dL * inv_rho;
            }
            const C beta = P / (P + C(2) * a.ph.mu);
            const C alpha = C(D + 2) / C(D) - rho * sCen[s0][CCS][tid] / P - a.ph.eta_over_mu;
            const C thetas = theta + alpha * theta * du;
            const C Ts = Tt - FF * inv_rho * inv_rho * C(0.5) * a.ph.inv_cv;
            const C e = a.ph.cv * Tt - a.ph.a * rho;
            const C es = a.ph.cv * Ts - a.ph.a * rho;
            const C eps_eq = e - C(0.5 * D) * theta;
            const C eps_st = es - C(0.5 * D) * thetas;
            AxisEq<C> eq[3], st[3];
            Axis3<C> pf[3];
            for (int d = 0; d < D; d++) {
                const C us = u[d] + F[d] * inv_rho;
                eq[d] = axis_eq(u[d], theta);
                st[d] = axis_eq(us, thetas);
                pf[d] = psi3(us, thetas + us * us + Phi[d]);
            }
            const C w_keep = C(1) - C(2) * beta, w_eq = C(3) * beta - C(1), w_st = C(1) - beta;
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const int ix = cx_of(i), iy = cy_of(i), iz = D == 3 ? cz_of(i) : 0;
                const C px = pick(eq[0].p, ix), py = pick(eq[1].p, iy);
                const C qx = pick(eq[0].q, ix), qy = pick(eq[1].q, iy);
                const C sx = pick(st[0].p, ix), sy = pick(st[1].p, iy);
                const C tx = pick(st[0].q, ix), ty = pick(st[1].q, iy);
                const C fsx = pick(pf[0], ix), fsy = pick(pf[1], iy);
                C feq, geqs, fst, gsts, sp;
                if (D == 2) {
                    feq = rho * px * py;
                    geqs = qx * py + px * qy;
                    fst = rho * fsx * fsy;
                    gsts = tx * sy + sx * ty;
                    sp = sx * sy;
                } else {
                    const C pz = pick(eq[2].p, iz), qz = pick(eq[2].q, iz);
                    const C sz = pick(st[2].p, iz), tz = pick(st[2].q, iz);
                    feq = rho * px * py * pz;
                    geqs = (qx * py + px * qy) * pz + px * py * qz;
                    fst = rho * fsx * fsy * pick(pf[2], iz);
                    gsts = (tx * sy + sx * ty) * sz + sx * sy * tz;
                    sp = sx * sy * sz;
                }
                const C geq = feq * eps_eq + C(0.5) * rho * geqs;
                C gst = rho * sp * eps_st + C(0.5) * rho * gsts;
                if (csq_of<D>(i) == 1) {
                    const C cq = ix ? (ix > 0 ? qc[0] : -qc[0]) : (iy ? (iy > 0 ? qc[1] : -qc[1]) : (iz > 0 ? qc[2] : -qc[2]));
                    gst += C(0.5) * cq;
                }
                fpost[i] = w_keep * fown[i] + w_eq * feq + w_st * fst;
                gpost[i] = w_keep * gown[i] + w_eq * geq + w_st * gst;
            }
            // stream: push to x + c_i of the other buffer (plane z + c_z wraps)
            const int gx = x0 + lx, gy = y0 + ly;
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const int ix = cx_of(i), iy = cy_of(i), iz = D == 3 ? cz_of(i) : 0;
                const T fe = S::enc(fpost[i], (C)a.ref.f[i]), ge = S::enc(gpost[i], (C)a.ref.g[i]);
                int dx[2], dy[2];
                const int nxd = push_axis(gx, ix, g.nx, g.clampx, dx);
                const int nyd = push_axis(gy, iy, g.ny, g.clampy, dy);
                int dz = z + iz;
                if (D == 3) dz = dz < 0 ? dz + nz : (dz >= nz ? dz - nz : dz);
                for (int aa = 0; aa < nxd; aa++)
                    for (int bb = 0; bb < nyd; bb++) {
                        const long long d = (long long)dx[aa] + (long long)g.nx * ((long long)dy[bb] + (long long)g.ny * dz);
                        a.fo[i * N + d] = fe;
                        a.go[i * N + d] = ge;
                    }
                // the stored value is what the next step reads: round the
                // moment sums through the storage form as well
                fpost[i] = S::load(&fe, 0, (C)a.ref.f[i]);
                gpost[i] = S::load(&ge, 0, (C)a.ref.g[i]);
            }
        }

        // -- moments of the pushed populations, per destination plane ------
        for (int cz = (D == 3 ? -1 : 0); cz <= (D == 3 ? 1 : 0); cz++) {
            C *acc = &sAcc[D == 3 ? zslot3(z + cz) : 0][0][0];
            for (int pass = 0; pass < 2; pass++) {  // pass 0: f (rho, j); pass 1: g (G)
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    const int i = k + (D == 3 ? 9 * (cz + 1) : 0);
                    sX[k][tid] = own ? (pass == 0 ? fpost[i] : gpost[i]) : C(0);
                }
                __syncthreads();
                for (int r = tid; r < TL::R1; r += NT) {
                    const int rx = r % TL::W1 - 1, ry = r / TL::W1 - 1;
                    if (rx > w || ry > h) continue;
                    const bool inx = rx >= 0 && rx < w, iny = ry >= 0 && ry < h;
                    const bool edge_x0 = g.clampx && inx && x0 + rx == 0;
                    const bool edge_x1 = g.clampx && inx && x0 + rx == g.nx - 1;
                    const bool edge_y0 = g.clampy && iny && y0 + ry == 0;
                    const bool edge_y1 = g.clampy && iny && y0 + ry == g.ny - 1;
                    C s0 = 0, sjx = 0, sjy = 0;
                    for (int k = 0; k < 9; k++) {
                        const int cxk = k % 3 - 1, cyk = k / 3 - 1;
                        // per-axis source options: normal (d - c) and, on a
                        // zero-gradient wall with c pointing inward, d itself
                        int xs[2], ys[2], nxs = 0, nys = 0;
                        if (rx - cxk >= 0 && rx - cxk < w) xs[nxs++] = rx - cxk;
                        if ((edge_x0 && cxk == 1) || (edge_x1 && cxk == -1)) xs[nxs++] = rx;
                        if (ry - cyk >= 0 && ry - cyk < h) ys[nys++] = ry - cyk;
                        if ((edge_y0 && cyk == 1) || (edge_y1 && cyk == -1)) ys[nys++] = ry;
                        for (int p = 0; p < nxs; p++)
                            for (int q = 0; q < nys; q++) {
                                const C v = sX[k][ys[q] * TX + xs[p]];
                                s0 += v;
                                if (pass == 0) {
                                    if (cxk) sjx += cxk > 0 ? v : -v;
                                    if (cyk) sjy += cyk > 0 ? v : -v;
                                }
                            }
                    }
                    if (pass == 0) {
                        acc[0 * TL::R1 + r] += s0;
                        acc[1 * TL::R1 + r] += sjx;
                        acc[2 * TL::R1 + r] += sjy;
                        if (D == 3 && cz) acc[3 * TL::R1 + r] += cz > 0 ? s0 : -s0;
                    } else {
                        acc[4 * TL::R1 + r] += s0;
                    }
                }
            }
        }
        __syncthreads();
        if (D == 3) {
            flush(z - 1);
        } else {
            flush(0);
        }
        __syncthreads();
    }
    if (D == 3) {
        flush(nz - 1);
        __syncthreads();
        flush(nz);
    }
}

// complete moments of a state (after init or set_populations): layer of
// plane z; the wrap layers and inbound slots are cleared separately
template <int D, class S, class TL>
__global__ void __launch_bounds__(BX) k_fused_moments(Grid g, RefPops ref, int nlayer, const typename S::T *fi,
                                                      const typename S::T *gi, typename S::C *Mc) {
    using C = typename S::C;
    constexpr int Q = Lattice<D>::Q;
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const long long c = cell_index<D>(g, x, y, z);
    C rho = 0, J[3] = {0, 0, 0}, G = 0;
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const C f = S::load(fi, i * g.N + c, (C)ref.f[i]);
        rho += f;
        if (cx_of(i)) J[0] += cx_of(i) > 0 ? f : -f;
        if (cy_of(i)) J[1] += cy_of(i) > 0 ? f : -f;
        if (D == 3 && cz_of(i)) J[2] += cz_of(i) > 0 ? f : -f;
        G += S::load(gi, i * g.N + c, (C)ref.g[i]);
    }
    const long long plane = (long long)g.nx * g.ny;
    const long long pc = (long long)x + (long long)g.nx * y;
    const int layer = layer_of<D>(z);
    C v[5] = {rho, J[0], J[1], J[2], G};
    for (int k = 0; k < 5; k++) Mc[((long long)k * nlayer + layer) * plane + pc] = v[k];
}

}  // namespace lbm
