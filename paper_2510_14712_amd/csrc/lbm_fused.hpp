// Single-pass fused step: every population is read once and written once per
// step (Section 3.2 and its flowchart: moments -> Korteweg force -> u, E, T,
// P, Phi, q^c -> attractors -> collide and stream).
//
// Streaming is done on the way in: the stored set is the post-collision one,
// a cell reads its arrived population i from x - c_i and writes its collided
// populations back to its own addresses, so every store is a full, aligned
// row and only the loads are shifted (one element along x at most).
//
// Decomposition.  A workgroup owns a TX x TY tile of (x, y) columns and one
// segment [z0, z1) of planes, which it marches through.  The non-local inputs
// of the collision are the moments of the post-streaming state: rho on the L1
// ball of radius 3 (Laplacian, then the Korteweg force at the face
// neighbours), j and G at the cell and its face neighbours.  Those moments are
// produced by the previous step: after colliding plane z the workgroup
// gathers the collided populations into per-thread moment accumulators of the
// cells they arrive at in the next step, in planes z-1, z, z+1: the thread's
// own cell and, for the low lanes of every wavefront, one cell of the one-cell
// ring around the tile.  A completed plane is written out as
//   Mc  tile cells: the tile's own part of the sum,
//   IN  ring cells: inbound slots of the neighbouring tile that owns the cell,
// and the planes z0-1 and z1 of a segment, which the neighbouring segments
// complete, go to two spill layers of Mc / IN.  k_fused_fixup then adds the
// inbound slots and spill layers into Mc (fixed order, one thread per cell),
// so the next step reads complete moments with one load per value.
//
// Per marching position z (rho(z+1..z+4) and L(z..z+2) in LDS, the
// populations of plane z in registers):
//   phase A  Laplacian L(z+3); fields u, T, P, h, Lambda, F, c_s^2 of plane
//            z+1 for the tile and its ring                         | barrier
//   phase B  collide plane z, store rho(z+5) (loaded at the top of the
//            iteration) over rho(z+1), store the collided set to the other
//            buffer, write its deviations to the exchange buffer, load the
//            arrived populations of plane z+1 (from planes z..z+2)  | barrier
//   gather   moment sums of planes z-1, z, z+1 for the tile and its ring;
//            plane z-1 is complete and is written out.
// One workgroup per compute unit for FP32 and FP64, two for the 16-bit forms
// (their exchange holds 16-bit codes): the registers hold the prefetched
// plane and the LDS the whole exchange, with two barriers per plane.
// Ghost cells of zero-gradient axes take the field of the clamped cell.
#pragma once

#include "lbm_kernels.hpp"
#include "lbm_mlp_device.hpp"

namespace lbm {

template <int TX_, int TY_> struct Tile {
    static constexpr int TX = TX_, TY = TY_, NT = TX_ * TY_;
    static constexpr int W3 = TX_ + 6, H3 = TY_ + 6, R3 = W3 * H3;
    static constexpr int W2 = TX_ + 4, H2 = TY_ + 4, R2 = W2 * H2;
    static constexpr int W1 = TX_ + 2, H1 = TY_ + 2, R1 = W1 * H1;
    // ring cells of a full tile = inbound slots per tile, layer and moment
    static constexpr int NR = 2 * TX_ + 2 * TY_ + 4;
    // perimeter cells of a full tile
    static constexpr int PMAX = 2 * TX_ + 2 * TY_ - 4;
    // inbound slot offsets: contributions coming from the left / right / ...
    // neighbour, stored at the receiving cell's row (FROM_L, FROM_R) or column
    static constexpr int FROM_L = 0, FROM_R = TY_, FROM_B = 2 * TY_, FROM_T = 2 * TY_ + TX_;
    static constexpr int FROM_BL = 2 * TY_ + 2 * TX_, FROM_BR = FROM_BL + 1, FROM_TL = FROM_BL + 2,
                         FROM_TR = FROM_BL + 3;
    static_assert(NR <= NT, "one thread per ring cell");
};

// first plane of z segment s (segments split nz as evenly as possible)
__host__ __device__ __forceinline__ int seg_lo(int s, int nz, int nseg) {
    return (int)(((long long)s * nz) / nseg);
}
// segment holding plane z
__host__ __device__ __forceinline__ int seg_of(int z, int nz, int nseg) {
    return (int)((((long long)z + 1) * nseg - 1) / nz);
}

template <class C, class T> struct FusedArgs {
    Grid g;
    Phys<C> ph;
    RefPops ref;
    int ntx, nty, nseg;  // tiles along x, y; z segments
    int nlay;            // layers of Mc / IN: nz planes + 2 spill layers per segment (D = 3), 1 (D = 2)
    int chunk;           // tiles per XCD in the remapped order, 0: identity order
    int pull;            // form of the input set: 0 arrived, 1 post-collision (read from x - c_i)
    // sums of the reference populations as hi + lo pairs (moment sums run
    // over deviations; the pair keeps the constant's rounding from biasing
    // every cell's mass the same way)
    C rsf_hi, rsf_lo, rsg_hi, rsg_lo;
    const T *fi;  // input pair buffer (f_i, g_i side by side)
    T *fo;        // output pair buffer
    const C *Mci;  // complete moments of the input state, [nlay][5][ny][nx]
    C *Mco, *INo;  // output: tile-own partial sums, inbound slots [nlay][tiles][5][NR]
    const C *INi;  // folding instances: the input state's inbound slots (Mci then holds partial sums)
    // surrogate equation of state (kernels built with MLP)
    const C *Tin;  // surrogate form: the network's T of every cell from k_eos_surrogate ([z][y][x])
    // which cells' network T passed the residual check: bit x % 32 of word
    // [z][y][x / 32] (accw words per row); the others take the exact inversion
    const unsigned *Acc;
    int accw;
    double inv_cv_d;  // 1 / c_v of the FP32 constant, for that inversion in FP64
};

// ring cell r of a w x h tile: bottom row, top row, left column, right column
__device__ __forceinline__ bool ring_pos(int r, int w, int h, int &rx, int &ry) {
    if (r < w + 2) { rx = r - 1; ry = -1; return true; }
    r -= w + 2;
    if (r < w + 2) { rx = r - 1; ry = h; return true; }
    r -= w + 2;
    if (r < h) { rx = -1; ry = r; return true; }
    r -= h;
    if (r < h) { rx = w; ry = r; return true; }
    return false;
}

// tile owning the ring cell (rx, ry) of tile (tx, ty) and the inbound slot
// there; false when the ring cell lies beyond a zero-gradient wall
template <class TL>
__device__ __forceinline__ bool ring_slot(const Grid &g, int ntx, int nty, int tx, int ty, int w, int h, int rx,
                                          int ry, int &tile, int &slot) {
    const int dx = rx < 0 ? -1 : (rx >= w ? 1 : 0);
    const int dy = ry < 0 ? -1 : (ry >= h ? 1 : 0);
    int nbx = tx + dx, nby = ty + dy;
    if (nbx < 0 || nbx >= ntx) {
        if (g.clampx) return false;
        nbx = nbx < 0 ? nbx + ntx : nbx - ntx;
    }
    if (nby < 0 || nby >= nty) {
        if (g.clampy) return false;
        nby = nby < 0 ? nby + nty : nby - nty;
    }
    if (dy == 0) slot = dx < 0 ? TL::FROM_R + ry : TL::FROM_L + ry;
    else if (dx == 0) slot = dy < 0 ? TL::FROM_T + rx : TL::FROM_B + rx;
    else if (dx < 0) slot = dy < 0 ? TL::FROM_TR : TL::FROM_BR;
    else slot = dy < 0 ? TL::FROM_TL : TL::FROM_BL;
    tile = nby * ntx + nbx;
    return true;
}

// sum of the inbound slots of tile-local cell (lx, ly) of a w x h tile; `in`
// points at the slots of one (tile, layer, moment)
template <class TL, class C>
__device__ __forceinline__ C inbound_sum(const C *in, int lx, int ly, int w, int h) {
    C v = 0;
    if (lx == 0) v += in[TL::FROM_L + ly];
    if (lx == w - 1) v += in[TL::FROM_R + ly];
    if (ly == 0) v += in[TL::FROM_B + lx];
    if (ly == h - 1) v += in[TL::FROM_T + lx];
    if (lx == 0 && ly == 0) v += in[TL::FROM_BL];
    if (lx == w - 1 && ly == 0) v += in[TL::FROM_BR];
    if (lx == 0 && ly == h - 1) v += in[TL::FROM_TL];
    if (lx == w - 1 && ly == h - 1) v += in[TL::FROM_TR];
    return v;
}

// inbound_sum for a tile of at least 2 x 2 cells, where a cell receives at
// most one side, one bottom/top and one corner contribution.  The three slots
// are loaded unconditionally (each index stays inside the slot array for any
// lx < w, ly < h) and absent ones replaced by zero, so the loads of a thread
// overlap instead of waiting one after another; the sum has inbound_sum's
// order (adding a zero leaves a value unchanged).
template <class TL, class C>
__device__ __forceinline__ C inbound_sum_2x2(const C *in, int lx, int ly, int w, int h) {
    const bool l = lx == 0, r = lx == w - 1, b = ly == 0, t = ly == h - 1;
    const C sh = in[(l ? TL::FROM_L : TL::FROM_R) + ly];
    const C sv = in[(b ? TL::FROM_B : TL::FROM_T) + lx];
    const C sc = in[TL::FROM_BL + (r ? 1 : 0) + (t ? 2 : 0)];
    const bool hs = l || r, vs = b || t;
    return ((hs ? sh : (C)0) + (vs ? sv : (C)0)) + ((hs && vs) ? sc : (C)0);
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

// gather source of destination offset d (tile-local) for velocity component
// c along an axis: d - c, or d itself on a zero-gradient wall when c points
// inward (pull with clamped index); -1 when the source is outside the tile
__device__ __forceinline__ int gather_src(int d, int c, int t0, int n, int clamp, int extent) {
    const int gd = t0 + d;
    const int s = (clamp && ((gd == 0 && c == 1) || (gd == n - 1 && c == -1))) ? d : d - c;
    return (s >= 0 && s < extent) ? s : -1;
}

// Inputs of one cell's collision (eqs. sh_vel_1, sh_temp_1, sh_T_1, qc_1,
// correction) gathered from the field pipeline.
template <class C> struct CollideIn {
    C rho, P, e, cs2;     // e: specific internal energy of the moments (eq. def_E)
    C u[3], F[3];
    C du;                 // divergence of u, central differences
    C dh[3], dT[3];       // central differences of h and T
    C L0[3], Lm[3], Lp[3];  // Lambda_a at the cell and its -/+ neighbours along a
};

// Relax f, g in place to the post-collision populations (eqs. fLBGK, gLBGK
// with the attractors of eqs. LBMeq, LBMstar, LBMeqG, LBMgstar).
template <int D, class C>
__device__ __forceinline__ void collide_cell(const Phys<C> &ph, const CollideIn<C> &in, C *f, C *g) {
    constexpr int Q = Lattice<D>::Q;
    const C rho = in.rho, P = in.P;
    const C inv_rho = fdiv(C(1), rho);
    const C theta = P * inv_rho;
    C qc[3], Phi[3], FF = 0;
    for (int d = 0; d < D; d++) {
        FF += in.F[d] * in.F[d];
        qc[d] = P * (in.dh[d] - ph.k_over_mu * in.dT[d]);
        C dL;
        if (in.u[d] > ph.sgn_eps) dL = in.L0[d] - in.Lm[d];
        else if (in.u[d] < -ph.sgn_eps) dL = in.Lp[d] - in.L0[d];
        else dL = C(0.5) * (in.Lp[d] - in.Lm[d]);
        Phi[d] = -dL * inv_rho;
    }
    const C beta = fdiv(P, P + C(2) * ph.mu);
    const C alpha = C(D + 2) / C(D) - fdiv(rho * in.cs2, P) - ph.eta_over_mu;
    const C thetas = theta + alpha * theta * in.du;
    // e(rho, T*) with T* = T - |F|^2 / (2 rho^2 c_v) (eq. sh_T_1): for van der
    // Waals e is linear in T, so e(rho, T*) = e - |F|^2 / (2 rho^2), taken
    // from the moments' own e (no round trip through T, which keeps the
    // attractor's energy consistent with the populations')
    const C e = in.e;
    const C es = e - FF * inv_rho * inv_rho * C(0.5);
    const C eps_eq = e - C(0.5 * D) * theta;
    const C eps_st = es - C(0.5 * D) * thetas;
    AxisEq<C> eq[3], st[3];
    Axis3<C> pf[3];
    for (int d = 0; d < D; d++) {
        const C us = in.u[d] + in.F[d] * inv_rho;
        eq[d] = axis_eq(in.u[d], theta);
        st[d] = axis_eq(us, thetas);
        pf[d] = psi3(us, thetas + us * us + Phi[d]);
    }
    const C w_keep = C(1) - C(2) * beta, w_eq = C(3) * beta - C(1), w_st = C(1) - beta;
    // The attractors enter only as w_eq (f^eq, g^eq) + w_st (f*, g*), and
    // they are products over the axes, so with r_x = 2 eps p_x + q_x
    //   w_eq f^eq_i = (w_eq rho) p_x p_y p_z
    //   w_eq g^eq_i = (w_eq rho / 2) [(r_x p_y + p_x q_y) p_z + p_x p_y q_z]
    // and likewise f*, g* with (s, t, eps*) and the f* factors pf: the x-y
    // products are formed once per (x, y) pair, the weights ride on the z
    // factors, and a direction costs a few multiply-adds.
    const C Af = w_eq * rho, Ag = C(0.5) * Af, Sf = w_st * rho, Sg = C(0.5) * Sf;
    C hq[3];
    for (int d = 0; d < 3; d++) hq[d] = d < D ? C(0.5) * w_st * qc[d] : C(0);  // w_st x the q^c term
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const int ix = cx_of(i), iy = cy_of(i), iz = D == 3 ? cz_of(i) : 0;
        const C px = pick(eq[0].p, ix), py = pick(eq[1].p, iy);
        const C qx = pick(eq[0].q, ix), qy = pick(eq[1].q, iy);
        const C sx = pick(st[0].p, ix), sy = pick(st[1].p, iy);
        const C tx = pick(st[0].q, ix), ty = pick(st[1].q, iy);
        const C rx = C(2) * eps_eq * px + qx, rsx = C(2) * eps_st * sx + tx;
        const C pxy = px * py, sxy = sx * sy, fxy = pick(pf[0], ix) * pick(pf[1], iy);
        const C cxy = rx * py + px * qy, dxy = rsx * sy + sx * ty;
        C fa, ga;  // w_eq f^eq + w_st f*,  w_eq g^eq + w_st g*
        if (D == 2) {
            fa = Af * pxy + Sf * fxy;
            ga = Ag * cxy + Sg * dxy;
        } else {
            const C pz = pick(eq[2].p, iz), qz = pick(eq[2].q, iz);
            const C sz = pick(st[2].p, iz), tz = pick(st[2].q, iz);
            fa = pxy * (Af * pz) + fxy * (Sf * pick(pf[2], iz));
            ga = cxy * (Ag * pz) + pxy * (Ag * qz) + dxy * (Sg * sz) + sxy * (Sg * tz);
        }
        if (csq_of<D>(i) == 1)
            ga += ix ? (ix > 0 ? hq[0] : -hq[0]) : (iy ? (iy > 0 ? hq[1] : -hq[1]) : (iz > 0 ? hq[2] : -hq[2]));
        f[i] = w_keep * f[i] + fa;
        g[i] = w_keep * g[i] + ga;
    }
}

// -- buffer access ------------------------------------------------------------
// The step addresses HBM through buffer resources (base address and byte size;
// word 3 = 0x00020000, the raw 32-bit data format of gfx9) with a 32-bit
// per-lane offset and a 32-bit uniform offset.  No per-lane 64-bit pointer is
// formed, so the compiler cannot hoist one per population into registers
// across the march, and the uniform part stays in scalar registers.  Accesses
// at or past the resource's size read zero and write nothing; the host keeps
// every resource below 2^31 bytes.
using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ Rsrc make_rsrc(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void buf_ld(Rsrc r, unsigned vo, unsigned so, float &v) {
    v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ __forceinline__ void buf_ld(Rsrc r, unsigned vo, unsigned so, double &v) {
    v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
__device__ __forceinline__ void buf_ld(Rsrc r, unsigned vo, unsigned so, uint16_t &v) {
    v = __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0);
}
__device__ __forceinline__ void buf_st(Rsrc r, unsigned vo, unsigned so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
}
__device__ __forceinline__ void buf_st(Rsrc r, unsigned vo, unsigned so, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, 0);
}
__device__ __forceinline__ void buf_st(Rsrc r, unsigned vo, unsigned so, uint16_t v) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, vo, so, 0);
}
// byte offset of an absent inbound slot: beyond every slot resource (each
// below 2^31 bytes), so the buffer load's range check returns zero without a
// memory access.  A cell's slot sum then needs no per-slot select and equals
// inbound_sum_2x2's, whose absent terms are zeros too.
constexpr unsigned SLOT_NONE = 0x80000000u;
// the (f_i, g_i) pair of one cell in one access
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// (vector elements are copied to scalars before __builtin_bit_cast: this
// compiler's bit_cast of an element expression such as v.y reads element 0)
__device__ __forceinline__ void pair_ld(Rsrc r, unsigned vo, unsigned so, float &f, float &g) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0);
    const unsigned lo = v.x, hi = v.y;
    f = __builtin_bit_cast(float, lo);
    g = __builtin_bit_cast(float, hi);
}
__device__ __forceinline__ void pair_ld(Rsrc r, unsigned vo, unsigned so, double &f, double &g) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0);
    f = __builtin_bit_cast(double, (u32x2){v.x, v.y});
    g = __builtin_bit_cast(double, (u32x2){v.z, v.w});
}
__device__ __forceinline__ void pair_ld(Rsrc r, unsigned vo, unsigned so, uint16_t &f, uint16_t &g) {
    const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0);
    f = (uint16_t)v;
    g = (uint16_t)(v >> 16);
}
// Population stores carry the non-temporal cache policy (aux bit 1): the post-collision set is read back only
// in the next step, after the whole lattice has streamed through L2, so keeping it there only evicts the
// neighbour planes the loads reuse.
__device__ __forceinline__ void pair_st(Rsrc r, unsigned vo, unsigned so, float f, float g) {
    __builtin_amdgcn_raw_buffer_store_b64((u32x2){__builtin_bit_cast(unsigned, f), __builtin_bit_cast(unsigned, g)}, r,
                                          vo, so, 2);
}
__device__ __forceinline__ void pair_st(Rsrc r, unsigned vo, unsigned so, double f, double g) {
    const u32x2 a = __builtin_bit_cast(u32x2, f), b = __builtin_bit_cast(u32x2, g);
    __builtin_amdgcn_raw_buffer_store_b128((u32x4){a.x, a.y, b.x, b.y}, r, vo, so, 2);
}
__device__ __forceinline__ void pair_st(Rsrc r, unsigned vo, unsigned so, uint16_t f, uint16_t g) {
    __builtin_amdgcn_raw_buffer_store_b32((unsigned)f | ((unsigned)g << 16), r, vo, so, 2);
}

// fields of one plane's cell kept in registers between marching positions
template <class C> struct CenterF {
    C rho, uz, F[3], P, cs2, T, e, h, Lz;
};

// FAST: every tile is full and the x, y axes are periodic (no zero-gradient
// wall in the tile plane); the per-lane wall and partial-tile cases then fold
// away at compile time.
// Surrogate equation of state, one pass per step ahead of the fused step.
// The network stands in for the caloric inversion T(rho, e) (Section 3.2,
// after eq. lbm_temp).  For every cell: rho, j, G from the complete moment
// side channel; the Korteweg force F = kappa rho grad(lap rho) from the rho
// stencil (central differences, ghosts of zero-gradient axes take the
// clamped cell's values, as in the fused step); u, E and e (eqs. def_u,
// def_E); the network's T_hat (both hidden layers on MFMA); the caloric residual
// |e(rho, T_hat) - e| / (c_v T_hat) against the threshold.  Writes T_hat of
// every cell and one bit per cell, set where T_hat passed; the fused step
// takes T_hat where the bit is set and the exact inversion of eq. lbm_temp,
// in FP64, where it is not (the fallback: one Newton step on e(rho, T) = e
// lands on it exactly for van der Waals).  A workgroup takes a 64 x 4 block
// of (x, y) columns (one row per wavefront) and marches through `zchunk`
// planes.  The rho of a 68 x 8 region
// (the block and two cells around it) is staged in LDS for four planes, the
// Laplacian of the 66 x 6 region in LDS for three, so that a plane costs one
// coalesced load of the region per thread-share instead of a load per stencil
// point; the region loads and the cell's j, G run two planes ahead of their use,
// so that their latency overlaps the network of the planes between.
//
// FOLD: the pass also completes the side channel, doing the perimeter part of
// k_fused_fixup's work.  Mc then holds the previous fused step's partial sums,
// complete already on the segment-end planes (the fix-up's end-plane launch
// runs between the fused step and the pass), and IN its inbound slots; every
// value the pass uses on another plane is completed on load with the fix-up's
// terms, order and rounding (a perimeter cell adds its slots), and the five
// complete moments of every cell go to Mco, which the next fused step reads.
// The fused step's tiles are the pass's 64 x 4 blocks; tiles of at least 2 x 2
// cells (the host falls back to the separate fix-up otherwise).
struct FoldArgs {
    const float *IN;  // inbound slots [nlay][tiles][5][NR]
    float *Mco;       // complete moments out, plane layers [nz][5][ny][nx]
    int ntx, nty, nseg;
};
template <int D, bool FOLD>
__global__ void __launch_bounds__(256, 2) k_eos_surrogate(Grid g, Phys<float> ph, const float *__restrict__ Mc,
                                                       float *__restrict__ Tout, const float *__restrict__ P,
                                                       const uint16_t *__restrict__ W2b,
                                                       const float *__restrict__ norm, float tol,
                                                       unsigned long long *count, int zchunk, FoldArgs fa,
                                                       unsigned long long *__restrict__ Acc) {
    using TL = Tile<64, 4>;
    constexpr int W2LD = 72;  // padded BF16 rows: conflict-free 16-byte A-operand reads
    constexpr int RW = 68, RN = RW * 8;   // rho region: x0 - 2 .. x0 + 65, y0 - 2 .. y0 + 5
    constexpr int LW = 66, LN = LW * 6;   // Laplacian region: x0 - 1 .. x0 + 64, y0 - 1 .. y0 + 4
    constexpr int KR = (RN + 255) / 256;  // region entries per thread
    constexpr int KL = (LN + 255) / 256;
    constexpr int NRP = D == 3 ? 4 : 1;   // planes held
    constexpr int NLP = D == 3 ? 3 : 1;
    __shared__ float sNet[mlp::OFF_W2 + 2 * mlp::H + 2];
    __shared__ __attribute__((aligned(16))) uint16_t sW2[mlp::H * W2LD];
    // rows padded to whole multiples of the block, so that every thread
    // stores its entries without a branch (the padding is never read)
    __shared__ float sRho[NRP][KR * 256];
    __shared__ float sLap[NLP][KL * 256];
    const int tid = threadIdx.x, lane = tid & 63;
    for (int r = tid; r < mlp::OFF_W2; r += 256) sNet[r] = P[r];
    for (int r = tid; r < 2 * mlp::H; r += 256) sNet[mlp::OFF_W2 + r] = P[mlp::OFF_B2 + r];  // b2, w3 row of T
    if (tid == 0) sNet[mlp::OFF_W2 + 2 * mlp::H] = P[mlp::OFF_B3];
    // W2 with its columns in the order of the layer-1 accumulator (see
    // forward_wave_l1mfma)
    for (int r = tid; r < mlp::H * mlp::H; r += 256) {
        const int m = r / mlp::H, k = r % mlp::H;
        sW2[m * W2LD + k] = W2b[m * mlp::H + mlp::w2_perm_col(k)];
    }
    const mlp::Net net{sNet + mlp::OFF_W1, sNet + mlp::OFF_B1, sW2, nullptr, sNet + mlp::OFF_W2,
                       sNet + mlp::OFF_W2 + mlp::H, sNet + mlp::OFF_W2 + 2 * mlp::H, W2LD};

    const int nx = g.nx, ny = g.ny, nz = D == 3 ? g.nz : 1;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    // the block's chunk of planes
    const int z0_blk = D == 3 ? blockIdx.z * zchunk : 0;
    const int z1_blk = D == 3 ? min(nz, z0_blk + zchunk) : 1;
    // lattice coordinate of any point near the block: wrapped (periodic) or
    // clamped (zero-gradient)
    auto ax = [](int v, int n, int clamp) {
        if (clamp) return v < 0 ? 0 : (v >= n ? n - 1 : v);
        v %= n;
        return v < 0 ? v + n : v;
    };
    const int x0 = blockIdx.x * 64, y0 = blockIdx.y * 4;
    const int x = x0 + lane, y = y0 + (tid >> 6);
    const bool act = x < nx && y < ny;  // other lanes evaluate a clamped cell and write nothing
    const int xc = min(x, nx - 1), yc = min(y, ny - 1);
    const unsigned oc = xc + nx * yc;
    // the thread's rho-region entries: lattice offsets in a plane
    unsigned roff[KR];
#pragma unroll
    for (int k = 0; k < KR; k++) {
        const int r = min(tid + 256 * k, RN - 1);
        roff[k] = (unsigned)(ax(x0 - 2 + r % RW, nx, g.clampx) + nx * ax(y0 - 2 + r / RW, ny, g.clampy));
    }
    // the thread's Laplacian-region entries: rho-region index of the point the
    // Laplacian is evaluated at (on a zero-gradient axis a ghost point is the
    // clamped cell, whose Laplacian it takes; on a periodic one the point itself)
    int lsrc[KL];
#pragma unroll
    for (int k = 0; k < KL; k++) {
        const int r = min(tid + 256 * k, LN - 1);
        const int lx = r % LW - 1, ly = r / LW - 1;
        const int ex = g.clampx ? ax(x0 + lx, nx, 1) - x0 : lx, ey = g.clampy ? ax(y0 + ly, ny, 1) - y0 : ly;
        lsrc[k] = (ey + 2) * RW + ex + 2;
    }
    const int ol = (yc - y0 + 1) * LW + (xc - x0 + 1);  // the cell in the Laplacian region
    const int orr = (yc - y0 + 2) * RW + (xc - x0 + 2);  // and in the rho region

    // FOLD: inbound-slot byte offsets (moment 0, within a layer) of a lattice
    // cell: its side, bottom/top and corner slot in its tile's array
    // (SLOT_NONE where the cell has none), and whether it lies on the tile's
    // left/right and bottom/top edge (as in inbound_sum)
    struct Slots {
        unsigned sh, sv, sc;
        bool hs, vs;
    };
    auto slots_of = [&](int xe, int ye) {
        const int tx = xe / TL::TX, ty = ye / TL::TY, lx = xe - tx * TL::TX, ly = ye - ty * TL::TY;
        const int w = min(TL::TX, g.nx - tx * TL::TX), h = min(TL::TY, g.ny - ty * TL::TY);
        const bool l = lx == 0, r = lx == w - 1, b = ly == 0, t = ly == h - 1;
        const unsigned base = (unsigned)(ty * fa.ntx + tx) * 5u * TL::NR;
        Slots o;  // byte offsets
        o.hs = l || r;
        o.vs = b || t;
        o.sh = o.hs ? (base + (unsigned)((l ? TL::FROM_L : TL::FROM_R) + ly)) * (unsigned)sizeof(float) : SLOT_NONE;
        o.sv = o.vs ? (base + (unsigned)((b ? TL::FROM_B : TL::FROM_T) + lx)) * (unsigned)sizeof(float) : SLOT_NONE;
        o.sc = o.hs && o.vs ? (base + (unsigned)(TL::FROM_BL + (r ? 1 : 0) + (t ? 2 : 0))) * (unsigned)sizeof(float)
                            : SLOT_NONE;
        return o;
    };
    Slots rsl[KR], osl;
    if (FOLD) {
#pragma unroll
        for (int k = 0; k < KR; k++) {
            const int r = min(tid + 256 * k, RN - 1);
            rsl[k] = slots_of(ax(x0 - 2 + r % RW, nx, g.clampx), ax(y0 - 2 + r / RW, ny, g.clampy));
        }
        osl = slots_of(xc, yc);
    }
    // the cell's row is a bottom or top row of its tile: uniform over the
    // wavefront (one row of the block, which is the tile)
    const bool row_perim = FOLD && __builtin_amdgcn_readfirstlane(osl.vs ? 1 : 0) != 0;
    const unsigned in_layer = (unsigned)(fa.ntx * fa.nty) * 5u * TL::NR;  // floats per IN layer

    // periodic plane index of q in [z0 - 2, z1 + 4) (conditional adds, no
    // division; set-up only: the march keeps wrapped plane counters, advanced
    // by inc, a compare and select)
    auto zw = [&](int q) {
        if (D != 3) return 0;
        while (q < 0) q += nz;
        while (q >= nz) q -= nz;
        return q;
    };
    auto inc = [&](int wq) { return D == 3 ? (wq + 1 == nz ? 0 : wq + 1) : 0; };
    auto rs = [](int q) { return D == 3 ? q & 3 : 0; };
    auto ls = [](int q) { return D == 3 ? (int)((unsigned)(q + 3 * 4096) % 3u) : 0; };  // q > -3 * 4096
    // One buffer resource per layer of the side channel (its 5 moments, the
    // moment picked by a uniform offset) and per layer of the inbound slots;
    // the host keeps 5 nx ny values below 2^31 bytes.  wq, lay: layer indices.
    const unsigned mc_bytes = 5u * plane * (unsigned)sizeof(float), ko = plane * (unsigned)sizeof(float);
    auto mcr = [&](int lay) { return make_rsrc(Mc + (size_t)lay * 5 * plane, mc_bytes); };
    auto inr = [&](int lay) { return make_rsrc(fa.IN + (size_t)lay * in_layer, in_layer * (unsigned)sizeof(float)); };
    // values loaded for a plane: the side channel's sums and (FOLD) the three
    // inbound slots of each
    constexpr int NS = FOLD ? 1 : 0;
    struct RhoIn {
        float m[KR];
        float s[NS ? KR : 1][3];
    };
    struct JgIn {
        float m[4];
        float s[NS ? 4 : 1][3];
    };
    // the moment's slot block is a uniform offset (no per-lane address arithmetic)
    auto load_slots = [&](Rsrc ri, const Slots &sl, int m, float (&v)[3]) {
        const unsigned mo = (unsigned)m * TL::NR * (unsigned)sizeof(float);
        buf_ld(ri, sl.sh, mo, v[0]);
        buf_ld(ri, sl.sv, mo, v[1]);
        buf_ld(ri, sl.sc, mo, v[2]);
    };
    // bit i: plane z0 - 2 + i (i < 64; a chunk spans zchunk + 6 planes, the
    // host keeps zchunk <= 58) is a segment's first or last plane, whose
    // moments the end-plane fix-up has completed; set up once per block from
    // the segment boundaries (one division each; a window longer than nz
    // holds a plane more than once)
    unsigned long long end_m = 0;
    if (D == 3 && FOLD) {
        const int q0 = z0_blk - 2, len = min(64, z1_blk + 4 - q0);
        auto mark = [&](int e) {
            int i = (e - q0) % nz;
            if (i < 0) i += nz;
            for (; i < len; i += nz) end_m |= 1ull << i;
        };
        int lo = 0;  // seg_lo(0)
        for (int sg = 0; sg < fa.nseg; sg++) {
            const int next = seg_lo(sg + 1, nz, fa.nseg);
            mark(lo);
            mark(next - 1);
            lo = next;
        }
    }
    // plane q (unwrapped) is a segment-end plane
    auto is_end = [&](int q) { return D == 3 && FOLD && ((end_m >> (q - (z0_blk - 2))) & 1ull) != 0; };
    // complete moment of a cell from its partial sum mc and slots sv: a
    // perimeter cell adds its slots (inbound_sum_2x2's terms, order and
    // rounding); the slots of an interior cell are absent and read as zero
    auto complete = [&](float mc, const float (&sv)[3], const Slots &sl) {
        return (sl.hs || sl.vs) ? mc + ((sv[0] + sv[1]) + sv[2]) : mc;
    };
    auto load_rho = [&](int wq, RhoIn &v) {
        const Rsrc r = mcr(wq);
#pragma unroll
        for (int k = 0; k < KR; k++) buf_ld(r, roff[k] * (unsigned)sizeof(float), 0u, v.m[k]);
        if (FOLD) {
            const Rsrc ri = inr(wq);
#pragma unroll
            for (int k = 0; k < KR; k++) load_slots(ri, rsl[k], 0, v.s[k]);
        }
    };
    // rho of plane q into its LDS ring slot, completed (FOLD) unless q is a
    // segment-end plane
    auto put_rho = [&](int q, const RhoIn &v) {
        const bool add = FOLD && !is_end(q);
#pragma unroll
        for (int k = 0; k < KR; k++) {
            float x = v.m[k];
            if (FOLD) x = add ? complete(x, v.s[k], rsl[k]) : x;
            sRho[rs(q)][tid + 256 * k] = x;
        }
    };
    auto load_jg = [&](int wq, JgIn &v) {
        const Rsrc r = mcr(wq);
#pragma unroll
        for (int k = 0; k < 4; k++) buf_ld(r, oc * (unsigned)sizeof(float), (unsigned)(k + 1) * ko, v.m[k]);
        if (FOLD) {
            const Rsrc ri = inr(wq);
            // a wavefront is one row of the tile: on an inner row only the two
            // edge lanes have a (side) slot, so the row loads that one alone
            if (row_perim) {
#pragma unroll
                for (int k = 0; k < 4; k++) load_slots(ri, osl, k + 1, v.s[k]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    buf_ld(ri, osl.sh, (unsigned)(k + 1) * TL::NR * (unsigned)sizeof(float), v.s[k][0]);
                    v.s[k][1] = v.s[k][2] = 0.0f;
                }
            }
        }
    };
    // Laplacian of plane q over the region (expression order as in the fused step)
    auto make_lap = [&](int q) {
        const float *rc = sRho[rs(q)], *rm = sRho[rs(q - 1)], *rp = sRho[rs(q + 1)];
#pragma unroll
        for (int k = 0; k < KL; k++) {
            const int c = lsrc[k];
            const float r0 = rc[c];
            float s = rc[c + 1] + rc[c - 1] - 2.0f * r0 + rc[c + RW] + rc[c - RW] - 2.0f * r0;
            if (D == 3) s += rp[c] + rm[c] - 2.0f * r0;
            sLap[ls(q)][tid + 256 * k] = s;
        }
    };

    const int z0 = z0_blk, z1 = z1_blk;
    unsigned long long n_fb = 0, n_eval = 0;
    // per-block constants: the input map x = 2 (v - lo) / (hi - lo) - 1 as
    // (v - lo) s - 1, the residual bound tol c_v, and 1 / c_v for the Newton step
    // (read once: the buffer stores of the march could alias them as far as
    // the compiler knows, which would reload them every plane)
    const float n0 = norm[0], n2 = norm[2], n4 = norm[4], n5 = norm[5];
    const float s0 = 2.0f / (norm[1] - n0), s1 = 2.0f / (norm[3] - n2);
    const float tol_cv = tol * ph.cv;
    // acceptance words [z][y][x / 64], one per wavefront (a row of the block)
    const unsigned nxb = (unsigned)(nx + 63) / 64u, acc_bytes = (unsigned)ny * nxb * 8u;
    const unsigned acc_off = ((unsigned)yc * nxb + blockIdx.x) * 8u;
    // prologue: rho of planes z0 - 2 .. z0 + 1 in LDS, the Laplacian of z0 - 1
    // and z0; rho of z0 + 2, z0 + 3 and j, G of z0, z0 + 1 in flight
    RhoIn va, vb;
    JgIn ja, jb;
    {
        RhoIn v[NRP];
        const int q0 = z0 - (D == 3 ? 2 : 0);
#pragma unroll
        for (int q = 0; q < NRP; q++) load_rho(zw(q0 + q), v[q]);
#pragma unroll
        for (int q = 0; q < NRP; q++) put_rho(q0 + q, v[q]);
    }
    if (D == 3) {
        load_rho(zw(z0 + 2), va);
        load_rho(zw(z0 + 3), vb);
    }
    load_jg(zw(z0), ja);
    if (D == 3) load_jg(zw(z0 + 1), jb);
    // plane counters of the march: rho to load (z + 4), j, G to load (z + 2),
    // and the plane itself
    int w_rho = zw(z0 + 4), w_jg = zw(z0 + 2), w_cur = zw(z0);
    __syncthreads();
    if (D == 3) make_lap(z0 - 1);
    make_lap(z0);
    __syncthreads();
    const mlp::L1Ops l1 = mlp::l1_operands(sNet + mlp::OFF_W1, sNet + mlp::OFF_B1);
    // plane z; vr: rho of plane z + 2 (then loaded with z + 4), jg: j, G of
    // plane z (then loaded with z + 2).  Two register sets take turns, so no
    // register with a load in flight is ever copied.
    auto plane_step = [&](int z, RhoIn &vr, JgIn &jg) {
        if (D == 3) {
            // rho of plane z + 2 into the slot of plane z - 2 (last read before
            // the previous plane's first barrier), the Laplacian of z + 1
            put_rho(z + 2, vr);
            load_rho(w_rho, vr);  // also past the chunk (unused there): the loads' wait counts stay exact
            w_rho = inc(w_rho);
            __syncthreads();
            make_lap(z + 1);
            __syncthreads();
        }
        const float r = sRho[rs(z)][orr];
        // j, G of the cell (completed: FOLD)
        float j[4];
        if (FOLD) {
            const bool add = !is_end(z);
#pragma unroll
            for (int k = 0; k < 4; k++) j[k] = add ? complete(jg.m[k], jg.s[k], osl) : jg.m[k];
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++) j[k] = jg.m[k];
        }
        if (D == 3) {
            load_jg(w_jg, jg);
            w_jg = inc(w_jg);
        }
        if (FOLD) {
            // the complete moments of the cell for the fused step (a lane
            // beyond the lattice writes its clamped cell's, the same values)
            const Rsrc ro = make_rsrc(fa.Mco + (size_t)w_cur * 5 * plane, mc_bytes);
            buf_st(ro, oc * (unsigned)sizeof(float), 0u, r);
#pragma unroll
            for (int k = 0; k < 4; k++) buf_st(ro, oc * (unsigned)sizeof(float), (unsigned)(k + 1) * ko, j[k]);
        }
        const float inv_rho = __builtin_amdgcn_rcpf(r);  // 1 ulp; feeds the network input and the residual
        const float *lc = sLap[ls(z)];
        float F[3];
        F[0] = ph.kappa * r * 0.5f * (lc[ol + 1] - lc[ol - 1]);
        F[1] = ph.kappa * r * 0.5f * (lc[ol + LW] - lc[ol - LW]);
        F[2] = D == 3 ? ph.kappa * r * 0.5f * (sLap[ls(z + 1)][ol] - sLap[ls(z - 1)][ol]) : 0.0f;
        float uF = 0.0f, u2 = 0.0f;
        for (int d = 0; d < 3; d++) {
            const float u = d < D ? (j[d] + 0.5f * F[d]) * inv_rho : 0.0f;
            uF += u * F[d];
            u2 += u * u;
        }
        const float E = (j[3] + 0.5f * uF) * inv_rho;
        const float e = E - 0.5f * u2;
        float yh[1];
        const float x0n = (r - n0) * s0 - 1.0f, x1n = (e - n2) * s1 - 1.0f;
        mlp::forward_wave_l1mfma<1>(x0n, x1n, net, l1, yh);
        float Th = yh[0] * n5 + n4;
        // relative residual |c_v T - a rho - e| / (c_v |T|) <= tol, without the
        // division; a NaN fails the test and takes the fallback
        const bool fb = !(fabsf(ph.cv * Th - ph.a * r - e) <= tol_cv * fabsf(Th));
        const unsigned long long accepted = __ballot(!fb);
        // every lane stores: a lane beyond the lattice evaluated the clamped
        // cell from the same inputs, so it writes the same values to it, and
        // a wavefront beyond the lattice's last row the same word as that
        // row's (no branch around the stores, which keeps the loads' wait
        // counts exact)
        buf_st(make_rsrc(Tout + (size_t)w_cur * plane, ko), oc * (unsigned)sizeof(float), 0u, Th);
        __builtin_amdgcn_raw_buffer_store_b64((u32x2){(unsigned)accepted, (unsigned)(accepted >> 32)},
                                              make_rsrc(Acc + (size_t)w_cur * ny * nxb, acc_bytes), acc_off, 0u, 0);
        w_cur = inc(w_cur);
        n_fb += __popcll(__ballot(fb && act));
        n_eval += __popcll(__ballot(act));
    };
    for (int z = z0; z < z1; z += 2) {
        plane_step(z, va, ja);
        if (z + 1 < z1) plane_step(z + 1, vb, jb);
    }
    if (lane == 0 && n_eval) {
        atomicAdd(&count[0], n_fb);
        atomicAdd(&count[1], n_eval);
    }
}

// Waves per SIMD asked of the compiler: two for the 16-bit forms without the
// surrogate (their LDS, with a 16-bit exchange, fits two workgroups per CU;
// measured 1.4x faster than one), one otherwise (the registers then hold the
// prefetched plane; for FP32, exchanging f and g in turn to fit two
// workgroups was slower).
template <class S, bool MLP> constexpr int fused_occupancy() { return sizeof(typename S::T) == 2 ? 2 : 1; }

template <int D, class S, class TL, bool MLP, bool FAST>
__global__ void __launch_bounds__(TL::NT, (fused_occupancy<S, MLP>())) k_fused(FusedArgs<typename S::C, typename S::T> a) {
    using C = typename S::C;
    using T = typename S::T;
    constexpr int Q = Lattice<D>::Q;
    constexpr int TX = TL::TX, TY = TL::TY, NT = TL::NT;
    constexpr int NRS = D == 3 ? 4 : 1;  // rho planes held in LDS
    constexpr int NLS = D == 3 ? 4 : 1;  // Laplacian planes
    constexpr int NFS = D == 3 ? 2 : 1;  // ring-field planes
    constexpr int XS = NT + 1;           // exchange row: NT cells, then a zero
    constexpr int NR3 = (TL::R3 + NT - 1) / NT;
    constexpr int NR2 = (TL::R2 + NT - 1) / NT;
    constexpr int NW = (NT + 63) / 64;  // wavefronts per workgroup
    // 32-sample halves of the surrogate needed for a wave's ring cells
    // ring fields on R1 (x, y neighbours of the collision): u_x, u_y, T, h,
    // Lambda_x, Lambda_y
    enum { RUX, RUY, RT, RH, RLX, RLY, NRF };
    __shared__ C sRho[NRS][TL::R3];
    __shared__ C sLap[NLS][TL::R2];
    __shared__ C sRing[NFS][NRF][TL::R1];
    using XT = typename S::X;
    constexpr int GROW = Q;          // first exchange row of g
    __shared__ XT sX[2 * Q][XS];  // exchange: deviations of the collided f (rows 0..Q-1) and g
    __shared__ C sRacc[D == 3 ? 3 : 1][5][TL::NR];  // moment sums of the ring destinations, by plane

    Grid g = a.g;
    if constexpr (FAST) {
        g.clampx = 0;
        g.clampy = 0;
    }
    // FOLD (the full-tile periodic instances with 16-bit storage and the
    // explicit EOS): the input side channel holds the previous step's
    // tile-own partial sums -- complete only on the segment-end planes, which
    // the fix-up's end-plane launch completes -- and INi its inbound slots.
    // Every moment read is completed on load with the fix-up's terms, order
    // and rounding (a perimeter cell adds its side, bottom/top and corner
    // slot), so the step needs no pass over the tiles' perimeter cells.  The
    // extra loads cost these instances less than the pass they replace; the
    // FP32 instance, already at the register limit, ran 30 % slower with them
    // and keeps the separate fix-up.
    constexpr bool FOLD = FAST && !MLP && sizeof(T) == 2;
    const long long N = g.N;
    const long long plane = (long long)g.nx * g.ny;
    const int tid = threadIdx.x;
    const int lane = tid & 63;

    // -- tile and segment of this workgroup ----------------------------------
    const int b = blockIdx.x;
    const int L = a.chunk ? (b & 7) * a.chunk + (b >> 3) : b;
    const int tx = L % a.ntx, ty = (L / a.ntx) % a.nty, seg = L / (a.ntx * a.nty);
    const int x0 = tx * TX, y0 = ty * TY;
    const int w = FAST ? TX : min(TX, g.nx - x0), h = FAST ? TY : min(TY, g.ny - y0);
    const int nz = g.nz;
    const int z0 = D == 3 ? seg_lo(seg, nz, a.nseg) : 0;
    const int z1 = D == 3 ? seg_lo(seg + 1, nz, a.nseg) : 1;

    // -- z-invariant per-thread set-up ---------------------------------------
    const int lx = tid % TX, ly = tid / TX;
    const bool own = FAST || (lx < w && ly < h);
    const int gx = x0 + min(lx, w - 1), gy = y0 + min(ly, h - 1);
    // per-lane offsets are unsigned 32-bit so that loads and stores take a
    // uniform 64-bit base plus a zero-extended lane offset
    const unsigned own_off = (unsigned)(gx + g.nx * gy);
    const int c3o = (ly + 3) * TL::W3 + lx + 3, c2o = (ly + 2) * TL::W2 + lx + 2, c1o = (ly + 1) * TL::W1 + lx + 1;

    // ring cell rid of this thread: ring cells are dealt round-robin over
    // the wavefronts (cell r to wave r mod NW, lane r / NW), so that every
    // wave carries the same share of ring work and the ring cells of a wave
    // sit in its low lanes
    const int rid = lane * NW + (tid >> 6);
    int rx = 0, ry = 0;
    const bool ring = ring_pos(rid, w, h, rx, ry);
    const int nring = 2 * (w + 2) + 2 * h;
    int rtile = 0, rslot = 0;
    const bool ring_dst = ring && ring_slot<TL>(g, a.ntx, a.nty, tx, ty, w, h, rx, ry, rtile, rslot);
    unsigned ring_off = own_off;
    int c3r = c3o, c2r = c2o, c1r = c1o;
    if (ring) {
        const int ex = axis_eff(x0, rx, g.nx, g.clampx), ey = axis_eff(y0, ry, g.ny, g.clampy);
        ring_off = (unsigned)(axis_global(x0, rx, g.nx, g.clampx) + g.nx * axis_global(y0, ry, g.ny, g.clampy));
        c3r = (ey + 3) * TL::W3 + ex + 3;
        c2r = (ey + 2) * TL::W2 + ex + 2;
        c1r = (ry + 1) * TL::W1 + rx + 1;
    }
    // rho of the R3 region: plane offsets of this thread's entries
    unsigned rho_off[NR3];
#pragma unroll
    for (int k = 0; k < NR3; k++) {
        const int r = min(tid + k * NT, TL::R3 - 1);
        rho_off[k] = (unsigned)(axis_global(x0, r % TL::W3 - 3, g.nx, g.clampx) +
                                g.nx * axis_global(y0, r / TL::W3 - 3, g.ny, g.clampy));
    }
    // FOLD: byte offsets (moment 0, within a layer) of the side, bottom/top
    // and corner slot of a lattice cell in its tile's slot array (SLOT_NONE
    // where it has none), and whether it lies on the tile's left/right and
    // bottom/top edge (full tiles)
    struct SlotRef {
        unsigned sh, sv, sc;
        bool hs, vs;
    };
    auto slot_ref = [&](int xe, int ye) {
        const int ttx = xe / TX, tty = ye / TY;
        const int ex = xe - ttx * TX, ey = ye - tty * TY;
        const bool l = ex == 0, r = ex == TX - 1, b = ey == 0, t = ey == TY - 1;
        const unsigned base = (unsigned)(tty * a.ntx + ttx) * 5u * TL::NR;
        SlotRef o;
        o.hs = l || r;
        o.vs = b || t;
        o.sh = o.hs ? (base + (unsigned)((l ? TL::FROM_L : TL::FROM_R) + ey)) * (unsigned)sizeof(C) : SLOT_NONE;
        o.sv = o.vs ? (base + (unsigned)((b ? TL::FROM_B : TL::FROM_T) + ex)) * (unsigned)sizeof(C) : SLOT_NONE;
        o.sc = o.hs && o.vs ? (base + (unsigned)(TL::FROM_BL + (r ? 1 : 0) + (t ? 2 : 0))) * (unsigned)sizeof(C)
                            : SLOT_NONE;
        return o;
    };
    SlotRef rho_ref[FOLD ? NR3 : 1], own_ref{}, ring_ref{};
    if constexpr (FOLD) {
#pragma unroll
        for (int k = 0; k < NR3; k++) {
            const int r = min(tid + k * NT, TL::R3 - 1);
            rho_ref[k] = slot_ref(axis_global(x0, r % TL::W3 - 3, g.nx, 0), axis_global(y0, r / TL::W3 - 3, g.ny, 0));
        }
        own_ref = slot_ref(gx, gy);
        ring_ref = ring ? slot_ref(axis_global(x0, rx, g.nx, 0), axis_global(y0, ry, g.ny, 0)) : own_ref;
    }
    // Laplacian on R2: R3 index of the evaluation point
    int lap_c[NR2];
#pragma unroll
    for (int k = 0; k < NR2; k++) {
        const int r = min(tid + k * NT, TL::R2 - 1);
        const int ei = axis_eff(x0, r % TL::W2 - 2, g.nx, g.clampx);
        const int ej = axis_eff(y0, r / TL::W2 - 2, g.ny, g.clampy);
        lap_c[k] = (ej + 3) * TL::W3 + ei + 3;
    }
    // gather sources of the own and the ring destination for the 9 in-plane
    // directions k = (c_x+1)+3(c_y+1): byte offsets into an exchange row (NT =
    // the zero entry), two 16-bit offsets per register
    unsigned so[5] = {0, 0, 0, 0, 0}, sr[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const int cx = k % 3 - 1, cy = k / 3 - 1;
        int sx = gather_src(lx, cx, x0, g.nx, g.clampx, w), sy = gather_src(ly, cy, y0, g.ny, g.clampy, h);
        const unsigned vo = (unsigned)((own && sx >= 0 && sy >= 0) ? sy * TX + sx : NT) * sizeof(XT);
        sx = gather_src(rx, cx, x0, g.nx, g.clampx, w);
        sy = gather_src(ry, cy, y0, g.ny, g.clampy, h);
        const unsigned vr = (unsigned)((ring_dst && sx >= 0 && sy >= 0) ? sy * TX + sx : NT) * sizeof(XT);
        so[k / 2] |= vo << (16 * (k & 1));
        sr[k / 2] |= vr << (16 * (k & 1));
    }
    static_assert((NT + 1) * sizeof(XT) < 65536, "16-bit exchange offsets");
    // streaming on the way in: the arrived population with velocity c comes
    // from x - c of the stored post-collision set (per axis: x and nx y
    // parts of the cell offset); the first step after an initialisation reads
    // the arrived set in place
    unsigned xs[3], ys[3];
#pragma unroll
    for (int c = -1; c <= 1; c++) {
        xs[c + 1] = (unsigned)pull_coord(gx, c, g.nx, g.clampx, a.pull);
        ys[c + 1] = (unsigned)(g.nx * pull_coord(gy, c, g.ny, g.clampy, a.pull));
    }

    // periodic plane index; the march only asks for planes within a few of
    // [0, nz), so conditional adds replace a division (one pass for nz >= 6)
    auto zwrap = [&](int p) {
        if (D != 3) return 0;
        while (p < 0) p += nz;
        while (p >= nz) p -= nz;
        return p;
    };
    auto s4 = [](int p) { return D == 3 ? p & 3 : 0; };
    auto s2 = [](int p) { return D == 3 ? p & 1 : 0; };
    auto s3 = [](int p) { return D == 3 ? (int)((unsigned)(p + 3 * 4096) % 3u) : 0; };  // p > -3 * 4096
    // side channel, layer-major Mc[layer][k][y][x]: one resource per layer
    // over its 5 moments, the moment selected by the uniform offset
    const unsigned mc_bytes = (unsigned)(5 * plane * (long long)sizeof(C));
    auto mc_layer = [&](const C *M, int layer) { return make_rsrc(M + (long long)layer * 5 * plane, mc_bytes); };
    // moment k at lane offset `off` (cells) of a layer's resource
    auto mom = [&](Rsrc r, int k, unsigned off) -> C {
        C v;
        buf_ld(r, off * (unsigned)sizeof(C), (unsigned)k * (unsigned)plane * (unsigned)sizeof(C), v);
        return v;
    };

    // reference populations in LDS (read where used, uniform), so that they
    // do not hold 2Q scalar registers through the march
    __shared__ C sRef[2 * Q];
    for (int r = tid; r < 2 * Q; r += NT) sRef[r] = (C)(r < Q ? a.ref.f[r] : a.ref.g[r - Q]);
    // zero columns of the exchange buffers, ring accumulators
    for (int r = tid; r < 2 * Q; r += NT) sX[r][NT] = S::xenc(C(0));
    for (int r = tid; r < (D == 3 ? 3 : 1) * 5 * TL::NR; r += NT) (&sRacc[0][0][0])[r] = C(0);

    // -- pipeline stages -----------------------------------------------------
    // FOLD: inbound slots of the input state, one resource per layer
    const unsigned in_layer = (unsigned)(a.ntx * a.nty) * 5u * TL::NR;
    auto in_in = [&](int layer) { return make_rsrc(a.INi + (size_t)layer * in_layer, in_layer * (unsigned)sizeof(C)); };
    auto ld_slots = [&](Rsrc ri, const SlotRef &sl, int m, C(&v)[3]) {
        const unsigned mo = (unsigned)m * TL::NR * (unsigned)sizeof(C);
        buf_ld(ri, sl.sh, mo, v[0]);
        buf_ld(ri, sl.sv, mo, v[1]);
        buf_ld(ri, sl.sc, mo, v[2]);
    };
    // the complete moment: inbound_sum_2x2's terms and order added to the
    // partial sum of a perimeter cell
    auto complete = [&](C mc, const C(&v)[3], const SlotRef &sl) {
        return (sl.hs || sl.vs) ? mc + ((v[0] + v[1]) + v[2]) : mc;  // absent slots read as zero
    };
    // segment-end planes hold complete moments already (the end-plane
    // fix-up); with segments of at least 6 planes the march's window
    // [z0 - 3, z1 + 5) meets no other segment's end plane
    const int zend_below = D == 3 ? zwrap(z0 - 1) : -1, zend_above = D == 3 ? zwrap(z1) : -1;
    auto is_end = [&](int p) {
        if (D != 3) return false;
        const int wp = zwrap(p);
        return wp == z0 || wp == z1 - 1 || wp == zend_below || wp == zend_above;
    };
    auto load_rho_regs = [&](int p, C *v, C(*vs)[3]) {
        const Rsrc r = mc_layer(a.Mci, zwrap(p));
#pragma unroll
        for (int k = 0; k < NR3; k++) v[k] = mom(r, 0, rho_off[k]);
        if constexpr (FOLD) {
            const Rsrc ri = in_in(zwrap(p));
#pragma unroll
            for (int k = 0; k < NR3; k++) ld_slots(ri, rho_ref[k], 0, vs[k]);
        }
    };
    auto store_rho = [&](int p, const C *v, const C(*vs)[3]) {
        C *dst = sRho[s4(p)];
        const bool add = FOLD && !is_end(p);
#pragma unroll
        for (int k = 0; k < NR3; k++) {
            C x = v[k];
            if constexpr (FOLD) x = add ? complete(x, vs[k], rho_ref[k]) : x;
            if (tid + k * NT < TL::R3) dst[tid + k * NT] = x;
        }
    };
    // surrogate form: acceptance words of the own and the ring cell of plane
    // p (loaded one plane ahead of the temperatures they select)
    const unsigned acc_row_bytes = (unsigned)a.accw * 4u;
    const unsigned acc_own = (unsigned)gy * acc_row_bytes + (unsigned)(gx >> 5) * 4u;
    unsigned acc_ring = acc_own;
    int bit_own = gx & 31, bit_ring = bit_own;
    if (MLP && ring) {
        const int rgx = axis_global(x0, rx, g.nx, g.clampx), rgy = axis_global(y0, ry, g.ny, g.clampy);
        acc_ring = (unsigned)rgy * acc_row_bytes + (unsigned)(rgx >> 5) * 4u;
        bit_ring = rgx & 31;
    }
    auto load_acc = [&](int p, unsigned &wo, unsigned &wr) {
        if constexpr (MLP) {
            const Rsrc rm = make_rsrc(a.Acc + (long long)zwrap(p) * g.ny * a.accw, (unsigned)g.ny * acc_row_bytes);
            wo = __builtin_amdgcn_raw_buffer_load_b32(rm, acc_own, 0u, 0);
            wr = __builtin_amdgcn_raw_buffer_load_b32(rm, acc_ring, 0u, 0);
        }
    };
    // j, G of plane p for the own and the ring cell; the surrogate form also
    // loads the network's T where the cell's acceptance bit (in wo / wr) is
    // set, and marks the cell accepted in jo[5] / jr[5] (1 or 0); a rejected
    // cell reads the plane's first entry instead, a line every cell of the
    // plane shares, so that no lane branches around its load
    auto load_jg = [&](int p, C *jo, C *jr, unsigned wo, unsigned wr) {
        const Rsrc r = mc_layer(a.Mci, zwrap(p));
#pragma unroll
        for (int k = 0; k < 4; k++) {
            jo[k] = mom(r, 1 + k, own_off);
            jr[k] = mom(r, 1 + k, ring_off);
        }
        if constexpr (MLP) {
            const bool ao = (wo >> bit_own) & 1u, ar = (wr >> bit_ring) & 1u;
            const Rsrc rt = make_rsrc(a.Tin + (long long)zwrap(p) * plane, (unsigned)(plane * (long long)sizeof(C)));
            buf_ld(rt, ao ? own_off * (unsigned)sizeof(C) : 0u, 0u, jo[4]);
            buf_ld(rt, ar ? ring_off * (unsigned)sizeof(C) : 0u, 0u, jr[4]);
            jo[5] = ao ? C(1) : C(0);
            jr[5] = ar ? C(1) : C(0);
        }
    };
    // FOLD: the slots of j, G of plane p for the own and the ring cell, and the
    // completion of a raw load_jg with them
    auto load_jg_slots = [&](int p, C(*os)[3], C(*rs)[3]) {
        if constexpr (FOLD) {
            const Rsrc ri = in_in(zwrap(p));
#pragma unroll
            for (int k = 0; k < 4; k++) {
                ld_slots(ri, own_ref, 1 + k, os[k]);
                ld_slots(ri, ring_ref, 1 + k, rs[k]);
            }
        }
    };
    auto complete_jg = [&](int p, C *jo, C *jr, const C(*os)[3], const C(*rs)[3]) {
        if constexpr (FOLD) {
            const bool add = !is_end(p);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                jo[k] = add ? complete(jo[k], os[k], own_ref) : jo[k];
                jr[k] = add ? complete(jr[k], rs[k], ring_ref) : jr[k];
            }
        }
    };
    auto make_lap = [&](int p) {
        const C *rc = sRho[s4(p)];
        const C *rm = sRho[s4(p - 1)];
        const C *rp = sRho[s4(p + 1)];
        C *dst = sLap[s4(p)];
#pragma unroll
        for (int k = 0; k < NR2; k++) {
            if (tid + k * NT >= TL::R2) continue;
            const int c = lap_c[k];
            const C r0 = rc[c];
            C s = rc[c + 1] + rc[c - 1] - C(2) * r0 + rc[c + TL::W3] + rc[c - TL::W3] - C(2) * r0;
            if (D == 3) s += rp[c] + rm[c] - C(2) * r0;
            dst[tid + k * NT] = s;
        }
    };

    // fields of logical plane p at one cell: R3 index c3, R2 index c2 of the
    // evaluation point, j, G (and T of the surrogate form) of the cell
    auto eval_cell = [&](int p, int c3, int c2, const C *jg, C u[3], C F[3], C &rho, C &Tt, C &ee, C &P, C &cs2,
                         C &hh, C Lam[3]) {
        const C *lc = sLap[s4(p)];
        const C *lm = sLap[s4(p - 1)];
        const C *lp = sLap[s4(p + 1)];
        rho = sRho[s4(p)][c3];
        const C inv_rho = fdiv(C(1), rho);
        C uF = 0, u2 = 0;
        F[0] = a.ph.kappa * rho * C(0.5) * (lc[c2 + 1] - lc[c2 - 1]);
        F[1] = a.ph.kappa * rho * C(0.5) * (lc[c2 + TL::W2] - lc[c2 - TL::W2]);
        F[2] = D == 3 ? a.ph.kappa * rho * C(0.5) * (lp[c2] - lm[c2]) : C(0);
        for (int d = 0; d < 3; d++) {
            u[d] = d < D ? (jg[d] + C(0.5) * F[d]) * inv_rho : C(0);
            uF += u[d] * F[d];
            u2 += u[d] * u[d];
        }
        const C E = (jg[3] + C(0.5) * uF) * inv_rho;
        const C e = E - C(0.5) * u2;
        if constexpr (MLP) {
            // the network's T where the residual check accepted it; elsewhere
            // the exact inversion of eq. lbm_temp, in FP64 (the fallback)
            Tt = jg[5] != C(0) ? jg[4]
                               : (C)(((double)e + (double)a.ph.a * (double)rho) * a.inv_cv_d);
        } else {
            Tt = (e + a.ph.a * rho) * a.ph.inv_cv;  // eq. lbm_temp
        }
        vdw_p_cs2(a.ph, rho, Tt, P, cs2);
        const C theta = P * inv_rho;
        for (int d = 0; d < 3; d++) Lam[d] = rho * u[d] * (u[d] * u[d] + C(3) * (theta - C(1.0 / 3.0)));
        hh = e + theta;
        ee = e;
    };
    // fields of plane p for the own cell (into cf) and the ring cell
    auto make_fields = [&](int p, const C *jo, const C *jr, CenterF<C> &cf) {
        C *rf = &sRing[s2(p)][0][0];
        {
            C u[3], F[3], rho, Tt, ee, P, cs2, hh, Lam[3];
            eval_cell(p, c3o, c2o, jo, u, F, rho, Tt, ee, P, cs2, hh, Lam);
            if (own) {
                rf[RUX * TL::R1 + c1o] = u[0];
                rf[RUY * TL::R1 + c1o] = u[1];
                rf[RT * TL::R1 + c1o] = Tt;
                rf[RH * TL::R1 + c1o] = hh;
                rf[RLX * TL::R1 + c1o] = Lam[0];
                rf[RLY * TL::R1 + c1o] = Lam[1];
            }
            cf.rho = rho;
            cf.uz = u[2];
            cf.F[0] = F[0];
            cf.F[1] = F[1];
            cf.F[2] = F[2];
            cf.P = P;
            cf.cs2 = cs2;
            cf.T = Tt;
            cf.e = ee;
            cf.h = hh;
            cf.Lz = Lam[2];
        }
        if ((tid >> 6) < nring) {  // wavefronts holding ring cells (lane 0 holds ring cell `wave`)
            C u[3], F[3], rho, Tt, ee, P, cs2, hh, Lam[3];
            eval_cell(p, c3r, c2r, jr, u, F, rho, Tt, ee, P, cs2, hh, Lam);
            if (ring) {
                rf[RUX * TL::R1 + c1r] = u[0];
                rf[RUY * TL::R1 + c1r] = u[1];
                rf[RT * TL::R1 + c1r] = Tt;
                rf[RH * TL::R1 + c1r] = hh;
                rf[RLX * TL::R1 + c1r] = Lam[0];
                rf[RLY * TL::R1 + c1r] = Lam[1];
            }
        }
    };

    // moment accumulators of the own destination in planes z-1, z, z+1
    // (registers); the ring destination's live in sRacc, slot p mod 3 for
    // plane p, touched only by the owning thread
    C acc[3][5];
#pragma unroll
    for (int q = 0; q < 3; q++)
#pragma unroll
        for (int k = 0; k < 5; k++) acc[q][k] = C(0);
    // inbound slots, layer-major: one resource per layer over every tile's
    // slots (the whole array may exceed what one resource addresses)
    auto in_rsrc = [&](int layer) { return make_rsrc(a.INo + (size_t)layer * in_layer, in_layer * (unsigned)sizeof(C)); };
    // write plane p (own: acc[0]) to `layer`, then clear its ring slot; the
    // reference sums enter once per cell, with the tile-own part of its plane
    auto flush = [&](int p, int layer) {
        if (own) {
            const Rsrc mo = mc_layer(a.Mco, layer);
            const bool plane_layer = D == 2 || layer < nz;
#pragma unroll
            for (int k = 0; k < 5; k++) {
                C v = acc[0][k];
                if (plane_layer && k == 0) v = (v + a.rsf_lo) + a.rsf_hi;
                if (plane_layer && k == 4) v = (v + a.rsg_lo) + a.rsg_hi;
                buf_st(mo, own_off * (unsigned)sizeof(C), (unsigned)k * (unsigned)plane * (unsigned)sizeof(C), v);
            }
        }
        if (ring) {
            C *ra = &sRacc[s3(p)][0][0];
            const Rsrc rIN = in_rsrc(layer);
#pragma unroll
            for (int k = 0; k < 5; k++) {
                if (ring_dst)
                    buf_st(rIN, ((unsigned)rtile * 5u * TL::NR + (unsigned)rslot) * (unsigned)sizeof(C),
                           (unsigned)(k * TL::NR * sizeof(C)), ra[k * TL::NR + rid]);
                ra[k * TL::NR + rid] = C(0);
            }
        }
    };
    auto shift_acc = [&]() {
#pragma unroll
        for (int k = 0; k < 5; k++) {
            acc[0][k] = acc[1][k];
            acc[1][k] = acc[2][k];
            acc[2][k] = C(0);
        }
    };
    // exchange: the deviations of the collided populations of the own cell
    auto xwrite = [&](const C *pp, int row0) {
#pragma unroll
        for (int i = 0; i < Q; i++) sX[row0 + i][tid] = S::xenc(pp[i]);
    };
    // gather of the directions with c_z = r - 1 (D = 3) of the set(s) in W
    // (1: f from rows i0 + k, 2: g from rows GROW + i0 + k)
    auto xgather = [&](auto W, int r, int z) {
        constexpr int w = decltype(W)::value;
        const int i0 = D == 3 ? 9 * r : 0;
        const char *X = (const char *)&sX[0][0];
        const int q = D == 3 ? r : 1;  // accumulator of plane z + c_z
        auto xv = [&](int row, const unsigned *src, int k) -> C {
            const unsigned off = (src[k / 2] >> (16 * (k & 1))) & 0xffffu;
            return S::xdec(*(const XT *)(X + (size_t)row * XS * sizeof(XT) + off));
        };
        // moment sums of the 3 x 3 in-plane directions k = (c_x + 1) + 3 (c_y + 1):
        // row sums first, then rho, j_y from the rows and j_x from the two
        // outer columns (14 additions instead of 21); no sum starts from zero
        auto sums = [&](const unsigned *src, C &s0, C &sx, C &sy, C &sg) {
            s0 = sx = sy = sg = C(0);
            if (w & 1) {
                C v[9];
#pragma unroll
                for (int k = 0; k < 9; k++) v[k] = xv(i0 + k, src, k);
                const C r0 = v[0] + v[1] + v[2], r1 = v[3] + v[4] + v[5], r2 = v[6] + v[7] + v[8];
                s0 = r0 + r1 + r2;
                sy = r2 - r0;
                sx = (v[2] + v[5] + v[8]) - (v[0] + v[3] + v[6]);
            }
            if (w & 2) {
                C t = xv(GROW + i0, src, 0);
#pragma unroll
                for (int k = 1; k < 9; k++) t += xv(GROW + i0 + k, src, k);
                sg = t;
            }
        };
        {
            C s0, sx, sy, sg;
            sums(so, s0, sx, sy, sg);
            if (w & 1) {
                acc[q][0] += s0;
                acc[q][1] += sx;
                acc[q][2] += sy;
                if (D == 3 && r != 1) acc[q][3] += r == 2 ? s0 : -s0;  // j_z: c_z s0, zero for c_z = 0
            }
            if (w & 2) acc[q][4] += sg;
        }
        if (ring) {
            C s0, sx, sy, sg;
            sums(sr, s0, sx, sy, sg);
            C *ra = &sRacc[s3(z + (D == 3 ? r - 1 : 0))][0][0];
            if (w & 1) {
                ra[0 * TL::NR + rid] += s0;
                ra[1 * TL::NR + rid] += sx;
                ra[2 * TL::NR + rid] += sy;
                if (D == 3 && r != 1) ra[3 * TL::NR + rid] += r == 2 ? s0 : -s0;
            }
            if (w & 2) ra[4 * TL::NR + rid] += sg;
        }
    };
    using WFG = std::integral_constant<int, 3>;

    // -- prologue: rho(z0-3 .. z0+4), L(z0-2 .. z0+2), fields of z0-1, z0 -----
    CenterF<C> Zc, Zm4;  // centre fields of plane z; plane z-1 (u_z, T, h, Lambda_z used)
    constexpr int NJ = MLP ? 6 : 4;  // j, G (and T, accepted flag of the surrogate form) per cell
    C jo[NJ], jr[NJ];
    unsigned wo = 0, wr = 0;  // acceptance words of the next plane whose j, G are loaded
    C jos[FOLD ? 4 : 1][3], jrs[FOLD ? 4 : 1][3];  // FOLD: slots of the j, G in flight
    C rvs[FOLD ? NR3 : 1][3];                       // FOLD: slots of the rho entries in flight
    // j, G of plane p complete on return (the prologue's loads)
    auto load_jg_now = [&](int p) {
        load_jg(p, jo, jr, wo, wr);
        load_jg_slots(p, jos, jrs);
        complete_jg(p, jo, jr, jos, jrs);
    };
    {
        C rv[NR3];
        if (D == 3) {
            // four rho slots: each plane is overwritten once its last reader
            // has passed a barrier
            for (int p = z0 - 3; p <= z0; p++) {
                load_rho_regs(p, rv, rvs);
                store_rho(p, rv, rvs);
            }
            __syncthreads();
            make_lap(z0 - 2);
            make_lap(z0 - 1);
            __syncthreads();
            load_rho_regs(z0 + 1, rv, rvs);
            store_rho(z0 + 1, rv, rvs);
            load_acc(z0 - 1, wo, wr);
            load_jg_now(z0 - 1);
            load_acc(z0, wo, wr);
            __syncthreads();
            make_lap(z0);
            __syncthreads();
            make_fields(z0 - 1, jo, jr, Zm4);
            __syncthreads();
            for (int p = z0 + 2; p <= z0 + 3; p++) {
                load_rho_regs(p, rv, rvs);
                store_rho(p, rv, rvs);
            }
            load_jg_now(z0);
            load_acc(z0 + 1, wo, wr);
            __syncthreads();
            make_lap(z0 + 1);
            make_lap(z0 + 2);
            __syncthreads();
            make_fields(z0, jo, jr, Zc);
            load_jg_now(z0 + 1);
            load_acc(z0 + 2, wo, wr);
            load_rho_regs(z0 + 4, rv, rvs);
            __syncthreads();
            store_rho(z0 + 4, rv, rvs);
        } else {
            load_rho_regs(0, rv, rvs);
            store_rho(0, rv, rvs);
            load_acc(0, wo, wr);
            load_jg_now(0);
            __syncthreads();
            make_lap(0);
            __syncthreads();
            make_fields(0, jo, jr, Zc);
        }
        __syncthreads();
    }

    // arrived populations of the own cell of plane p into f, g (loaded one
    // position ahead, so that their latency overlaps the exchange and the
    // field pipeline)
    C f[Q], gq[Q];
    auto load_pops = [&](int p) {
        // one resource per source plane (c_z = -1, 0, +1 read planes p + 1,
        // p, p - 1 of the pulled set) over its Q nx ny pairs; uniform offset
        // of direction i, lane offset of the source cell
        constexpr unsigned PB = 2 * sizeof(T);  // bytes of an (f, g) pair
        const unsigned pbytes = (unsigned)((long long)Q * plane * PB);
        Rsrc rp[3];
#pragma unroll
        for (int c = 0; c < (D == 3 ? 3 : 1); c++) {
            const int ps = D == 3 ? zwrap(p - a.pull * (c - 1)) : 0;
            rp[c] = make_rsrc(a.fi + 2 * (long long)ps * Q * plane, pbytes);
        }
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const int c = D == 3 ? cz_of(i) + 1 : 0;
            const unsigned so = (unsigned)i * (unsigned)plane * PB;
            const unsigned vo = (xs[cx_of(i) + 1] + ys[cy_of(i) + 1]) * PB;
            T rawf, rawg;
            pair_ld(rp[c], vo, so, rawf, rawg);
            f[i] = S::load(&rawf, 0, sRef[i]);
            gq[i] = S::load(&rawg, 0, sRef[Q + i]);
        }
    };
    load_pops(z0);

    for (int z = z0; z < z1; z++) {
        // -- prefetch of rho(z+5) and j, G(z+2); phase A: L(z+3), fields of
        //    plane z+1 ------------------------------------------------------------
        C rv[NR3], jon[NJ], jrn[NJ];
        CenterF<C> Zp;
        __builtin_amdgcn_s_setprio(2);  // raised outside the collision (see phase B)
        if (D == 3) {
            load_rho_regs(z + 5, rv, rvs);
            load_jg(z + 2, jon, jrn, wo, wr);
            load_acc(z + 3, wo, wr);
            make_lap(z + 3);
            __builtin_amdgcn_s_setprio(0);  // arithmetic, as the collision (see phase B)
            make_fields(z + 1, jo, jr, Zp);
            __builtin_amdgcn_s_setprio(2);
            __syncthreads();
        }

        // -- phase B: collide the own cell of plane z ---------------------------
        // Wavefront priority: the collision and the fields of the next plane,
        // long stretches of arithmetic with no memory access or barrier, run
        // at the base priority; the rest of the iteration (loads, LDS
        // stencils and exchange, the two barriers) at a raised one.  Two
        // workgroups share a compute unit in the 16-bit forms, so a wavefront
        // in its load and barrier phases takes precedence over the other
        // workgroup's arithmetic, which fills the gaps (BF16 + surrogate at
        // 512^3: k_fused 9.16 -> 8.55 ms; loads alone raised 9.10, phase A
        // 8.91, all but the collision 8.60)
        __builtin_amdgcn_s_setprio(0);
        {
            const C *rf = &sRing[s2(z)][0][0];
            CollideIn<C> in;
            in.rho = Zc.rho;
            in.P = Zc.P;
            in.e = Zc.e;
            in.cs2 = Zc.cs2;
            in.u[0] = rf[RUX * TL::R1 + c1o];
            in.u[1] = rf[RUY * TL::R1 + c1o];
            in.u[2] = Zc.uz;
            in.F[0] = Zc.F[0];
            in.F[1] = Zc.F[1];
            in.F[2] = Zc.F[2];
            in.du = C(0.5) * (rf[RUX * TL::R1 + c1o + 1] - rf[RUX * TL::R1 + c1o - 1]) +
                    C(0.5) * (rf[RUY * TL::R1 + c1o + TL::W1] - rf[RUY * TL::R1 + c1o - TL::W1]);
            in.dh[0] = C(0.5) * (rf[RH * TL::R1 + c1o + 1] - rf[RH * TL::R1 + c1o - 1]);
            in.dh[1] = C(0.5) * (rf[RH * TL::R1 + c1o + TL::W1] - rf[RH * TL::R1 + c1o - TL::W1]);
            in.dT[0] = C(0.5) * (rf[RT * TL::R1 + c1o + 1] - rf[RT * TL::R1 + c1o - 1]);
            in.dT[1] = C(0.5) * (rf[RT * TL::R1 + c1o + TL::W1] - rf[RT * TL::R1 + c1o - TL::W1]);
            in.L0[0] = rf[RLX * TL::R1 + c1o];
            in.Lm[0] = rf[RLX * TL::R1 + c1o - 1];
            in.Lp[0] = rf[RLX * TL::R1 + c1o + 1];
            in.L0[1] = rf[RLY * TL::R1 + c1o];
            in.Lm[1] = rf[RLY * TL::R1 + c1o - TL::W1];
            in.Lp[1] = rf[RLY * TL::R1 + c1o + TL::W1];
            if (D == 3) {
                in.du += C(0.5) * (Zp.uz - Zm4.uz);
                in.dT[2] = C(0.5) * (Zp.T - Zm4.T);
                in.dh[2] = C(0.5) * (Zp.h - Zm4.h);
                in.L0[2] = Zc.Lz;
                in.Lm[2] = Zm4.Lz;
                in.Lp[2] = Zp.Lz;
            } else {
                in.dT[2] = in.dh[2] = in.L0[2] = in.Lm[2] = in.Lp[2] = C(0);
            }
            collide_cell<D>(a.ph, in, f, gq);
        }
        if (D == 3) {
            store_rho(z + 5, rv, rvs);
#pragma unroll
            for (int k = 0; k < NJ; k++) {
                jo[k] = jon[k];
                jr[k] = jrn[k];
            }
        }
        __builtin_amdgcn_s_setprio(2);
        // -- store the post-collision set at the cell itself (the next step
        //    streams it on the way in); the moment sums of the next step use
        //    the stored values (as deviations) --------------------------------
        {
            constexpr unsigned PB = 2 * sizeof(T);  // bytes of an (f, g) pair
            const long long pb = 2 * (long long)(D == 3 ? z : 0) * Q * plane;
            const Rsrc ro = make_rsrc(a.fo + pb, (unsigned)((long long)Q * plane * PB));
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const C rf_i = sRef[i], rg_i = sRef[Q + i];
                T fe, ge;
                S::enc2(f[i], rf_i, gq[i], rg_i, fe, ge);
                f[i] = S::dev(&fe, 0, rf_i);
                gq[i] = S::dev(&ge, 0, rg_i);
                if (own) pair_st(ro, own_off * PB, (unsigned)i * (unsigned)plane * PB, fe, ge);
            }
        }

        // -- exchange, then the next position's populations, then the gather
        //    by c_z --------------------------------------------------------------
        auto rounds = [&](auto W) {
            if (D == 3) {
                xgather(W, 0, z);
                xgather(W, 1, z);
                xgather(W, 2, z);
            } else {
                xgather(W, 0, 0);
            }
        };
        xwrite(f, 0);
        xwrite(gq, GROW);
        if (D == 3 && z + 1 < z1) load_pops(z + 1);
        if (D == 3) load_jg_slots(z + 2, jos, jrs);  // FOLD (live across the gather, not the collision)
        __syncthreads();
        rounds(WFG{});
        if (D == 3) {
            flush(z - 1, z == z0 ? nz + 2 * seg : z - 1);  // plane z-1 is complete
            shift_acc();
            complete_jg(z + 2, jo, jr, jos, jrs);  // FOLD: j, G of plane z+2 (moved into jo, jr above)
            Zm4 = Zc;
            Zc = Zp;
        } else {
            // accumulator 1 holds plane 0
#pragma unroll
            for (int k = 0; k < 5; k++) acc[0][k] = acc[1][k];
            flush(0, 0);
        }
    }
    if (D == 3) {
        flush(z1 - 1, z1 - 1);
        shift_acc();
        flush(z1, nz + 2 * seg + 1);
    }
}

// Completes the moments of the output state: adds the inbound slots of tile
// edge cells and the spill layers of the segment end planes into Mc (own
// layers).  mode 0: perimeter cells of tiles in planes that are not segment
// ends, grid (ceil(tiles * PMAX / BX), nz); mode 1 (D = 3): every cell of the
// first and last plane of each segment, grid (ceil(nx ny / BX), 2 nseg).
template <int D, class TL, class C>
__global__ void __launch_bounds__(BX) k_fused_fixup(Grid g, int ntx, int nty, int nseg, int mode,
                                                    C *__restrict__ Mc, const C *__restrict__ IN) {
    // 32-bit index arithmetic throughout (tiles x perimeter slots, planes and
    // layers all fit); the z plane and its segment are uniform per block
    const int nz = g.nz;
    int z, s = 0;
    int gxv, gyv;
    if (mode == 0) {
        z = blockIdx.y;
        if (D == 3) {
            s = seg_of(z, nz, nseg);
            if (z == seg_lo(s, nz, nseg) || z == seg_lo(s + 1, nz, nseg) - 1) return;
        }
        const unsigned idx = blockIdx.x * (unsigned)BX + threadIdx.x;
        const unsigned tile = idx / (unsigned)TL::PMAX;  // compile-time divisor
        const int q = (int)(idx - tile * (unsigned)TL::PMAX);
        if (tile >= (unsigned)(ntx * nty)) return;
        const int tx = (int)(tile % (unsigned)ntx), ty = (int)(tile / (unsigned)ntx);
        const int w = min(TL::TX, g.nx - tx * TL::TX), h = min(TL::TY, g.ny - ty * TL::TY);
        int lx, ly;
        if (w == 1 || h == 1) {
            if (q >= w * h) return;
            lx = q % w;
            ly = q / w;
        } else {
            if (q >= 2 * w + 2 * h - 4) return;
            if (q < w) { lx = q; ly = 0; }
            else if (q < 2 * w) { lx = q - w; ly = h - 1; }
            else if (q < 2 * w + h - 2) { lx = 0; ly = 1 + q - 2 * w; }
            else { lx = w - 1; ly = 1 + q - (2 * w + h - 2); }
        }
        gxv = tx * TL::TX + lx;
        gyv = ty * TL::TY + ly;
    } else {
        s = blockIdx.y >> 1;
        const int zlo = seg_lo(s, nz, nseg), zhi = seg_lo(s + 1, nz, nseg) - 1;
        if ((blockIdx.y & 1) && zhi == zlo) return;
        z = (blockIdx.y & 1) ? zhi : zlo;
        const unsigned c = blockIdx.x * (unsigned)BX + threadIdx.x;
        if (c >= (unsigned)g.nx * (unsigned)g.ny) return;
        gxv = (int)(c % (unsigned)g.nx);
        gyv = (int)(c / (unsigned)g.nx);
    }
    const int tx = gxv / TL::TX, ty = gyv / TL::TY;
    const int lx = gxv - tx * TL::TX, ly = gyv - ty * TL::TY;
    const int w = min(TL::TX, g.nx - tx * TL::TX), h = min(TL::TY, g.ny - ty * TL::TY);
    const unsigned tile = (unsigned)(ty * ntx + tx);
    const unsigned plane = (unsigned)g.nx * (unsigned)g.ny;
    const unsigned cell = (unsigned)gxv + (unsigned)g.nx * (unsigned)gyv;
    // layer-major side channel: one layer's moments lie within 5 nx ny values
    auto mc = [&](int layer, int k) -> C & { return Mc[(size_t)(layer * 5 + k) * plane + cell]; };
    // inbound slots, layer-major [nlay][tiles][5][NR]
    const unsigned ntile = (unsigned)(ntx * nty);
    auto in = [&](int layer, int k) {
        return IN + (size_t)layer * ntile * 5u * TL::NR + ((size_t)tile * 5u + (unsigned)k) * TL::NR;
    };
    if (D == 3 && mode == 1) {
        const int zlo = seg_lo(s, nz, nseg), zhi = seg_lo(s + 1, nz, nseg) - 1;
        const int lay_hi = nz + 2 * ((s + nseg - 1) % nseg) + 1;  // plane z0 of segment s, from segment s-1
        const int lay_lo = nz + 2 * ((s + 1) % nseg);             // plane z1-1 of segment s, from segment s+1
        for (int k = 0; k < 5; k++) {
            C v = mc(z, k) + inbound_sum<TL>(in(z, k), lx, ly, w, h);
            if (z == zlo) v += mc(lay_hi, k) + inbound_sum<TL>(in(lay_hi, k), lx, ly, w, h);
            if (z == zhi) v += mc(lay_lo, k) + inbound_sum<TL>(in(lay_lo, k), lx, ly, w, h);
            mc(z, k) = v;
        }
    } else {
        // all loads of the cell first, then the stores: one memory round trip
        // per thread instead of one per moment
        C v[5];
#pragma unroll
        for (int k = 0; k < 5; k++) v[k] = mc(z, k);
        if (w >= 2 && h >= 2) {
#pragma unroll
            for (int k = 0; k < 5; k++) v[k] += inbound_sum_2x2<TL>(in(z, k), lx, ly, w, h);
        } else {
#pragma unroll
            for (int k = 0; k < 5; k++) v[k] += inbound_sum<TL>(in(z, k), lx, ly, w, h);
        }
#pragma unroll
        for (int k = 0; k < 5; k++) mc(z, k) = v[k];
    }
}

// Complete moments of a stored state (after init or set_populations) in the
// plane layers of Mc, summed in exactly the order, grouping and rounding of
// the fused step's gather and fix-up: deviation sums per source tile and
// segment, accumulated round by round (c_z = +1, 0, -1), the reference sums
// added to the tile-own part, then the inbound and spill parts in fix-up
// order.  A state restored from its populations therefore continues bitwise
// like the run that produced it.  The stored set may be in either form
// (`pull`, see arrived_index).  One thread per cell.
template <int D, class S, class TL>
__global__ void __launch_bounds__(BX) k_fused_moments(Grid g, RefPops ref, typename S::C rsf_hi,
                                                      typename S::C rsf_lo, typename S::C rsg_hi, typename S::C rsg_lo,
                                                      int ntx, int nty, int nseg, int nlay, const typename S::T *fi,
                                                      const typename S::T *gi, typename S::C *Mc, int pull) {
    using C = typename S::C;
    const int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    const int nz = g.nz;
    const int tx = x / TL::TX, ty = y / TL::TY;
    const int lx = x - tx * TL::TX, ly = y - ty * TL::TY;
    const int x0 = tx * TL::TX, y0 = ty * TL::TY;
    const int w = min(TL::TX, g.nx - x0), h = min(TL::TY, g.ny - y0);
    int z0 = 0, z1 = 1;
    if (D == 3) {
        const int s = seg_of(z, nz, nseg);
        z0 = seg_lo(s, nz, nseg);
        z1 = seg_lo(s + 1, nz, nseg);
    }
    const long long cell = cell_index<D>(g, x, y, z);
    // acc[class][group][moment]: class 0 sources in the own segment, 1 in
    // plane z0-1 (segment below), 2 in plane z1 (segment above); group =
    // source tile relative to the cell's tile, (oy + 1) * 3 + (ox + 1)
    C acc[3][9][5];
    for (int c = 0; c < 3; c++)
        for (int q = 0; q < 9; q++)
            for (int k = 0; k < 5; k++) acc[c][q][k] = C(0);
    for (int r = 0; r < (D == 3 ? 3 : 1); r++) {
        const int cz = D == 3 ? 1 - r : 0;  // the march meets sources at z-1 first
        int cls = 0;
        if (D == 3) cls = z - cz < z0 ? 1 : (z - cz >= z1 ? 2 : 0);
        C v[9], vg[9];
        int src[9];
        for (int k = 0; k < 9; k++) {
            const int cx = k % 3 - 1, cy = k / 3 - 1;
            const int i = k + (D == 3 ? 9 * (cz + 1) : 0);
            // source along each axis in tile-local coordinates (d - c, or d
            // itself on a zero-gradient wall when c points inward)
            const int sxl = (g.clampx && ((x == 0 && cx == 1) || (x == g.nx - 1 && cx == -1))) ? lx : lx - cx;
            const int syl = (g.clampy && ((y == 0 && cy == 1) || (y == g.ny - 1 && cy == -1))) ? ly : ly - cy;
            src[k] = ((syl < 0 ? -1 : (syl >= h ? 1 : 0)) + 1) * 3 + (sxl < 0 ? -1 : (sxl >= w ? 1 : 0)) + 1;
            const long long pi = arrived_index<D>(g, i, x, y, D == 3 ? z : 0, pull);
            v[k] = S::dev(fi, pi, (C)ref.f[i]);
            vg[k] = S::dev(gi, pi, (C)ref.g[i]);
        }
        // per source tile, the gather's sums over its share of the 3 x 3
        // directions (the others read as zero), in the gather's order
        for (int q = 0; q < 9; q++) {
            C a[9], b[9];
            for (int k = 0; k < 9; k++) {
                a[k] = src[k] == q ? v[k] : C(0);
                b[k] = src[k] == q ? vg[k] : C(0);
            }
            const C r0 = a[0] + a[1] + a[2], r1 = a[3] + a[4] + a[5], r2 = a[6] + a[7] + a[8];
            const C s0 = r0 + r1 + r2;
            C sg = b[0];
            for (int k = 1; k < 9; k++) sg += b[k];
            acc[cls][q][0] += s0;
            acc[cls][q][1] += (a[2] + a[5] + a[8]) - (a[0] + a[3] + a[6]);
            acc[cls][q][2] += r2 - r0;
            if (cz != 0) acc[cls][q][3] += cz > 0 ? s0 : -s0;
            acc[cls][q][4] += sg;
        }
    }
    // inbound part of one class in the order of the fix-up pass
    auto inbound = [&](int c, int k) -> C {
        C v = 0;
        if (lx == 0) v += acc[c][3][k];
        if (lx == w - 1) v += acc[c][5][k];
        if (ly == 0) v += acc[c][1][k];
        if (ly == h - 1) v += acc[c][7][k];
        if (lx == 0 && ly == 0) v += acc[c][0][k];
        if (lx == w - 1 && ly == 0) v += acc[c][2][k];
        if (lx == 0 && ly == h - 1) v += acc[c][6][k];
        if (lx == w - 1 && ly == h - 1) v += acc[c][8][k];
        return v;
    };
    const bool seg_end = D == 3 && (z == z0 || z == z1 - 1);
    const bool edge = lx == 0 || lx == w - 1 || ly == 0 || ly == h - 1;
    const long long plane = (long long)g.nx * g.ny;
    const long long pc = (long long)x + (long long)g.nx * y;
    for (int k = 0; k < 5; k++) {
        C v = acc[0][4][k];
        if (k == 0) v = (v + rsf_lo) + rsf_hi;
        if (k == 4) v = (v + rsg_lo) + rsg_hi;
        if (seg_end || edge) v = v + inbound(0, k);
        if (seg_end) {
            if (z == z0) v += acc[1][4][k] + inbound(1, k);
            if (z == z1 - 1) v += acc[2][4][k] + inbound(2, k);
        }
        Mc[((long long)(D == 3 ? z : 0) * 5 + k) * plane + pc] = v;
    }
}

}  // namespace lbm
