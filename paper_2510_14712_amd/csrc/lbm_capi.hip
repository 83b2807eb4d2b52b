// C ABI of the non-ideal DDF lattice Boltzmann library (declared in lbm.h):
// context management, launches of the step kernels, moments, population
// access, conservation sums and the stand-alone codec.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>

#include "lbm.h"
#include "lbm_internal.hpp"
#include <algorithm>
#include <type_traits>

using namespace lbm;

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions: per-block partials (wavefront shuffles, then
// LDS), then a single block summing the partials in block order.
// ---------------------------------------------------------------------------
namespace lbm {
constexpr int RED_BLOCK = 256;
constexpr int RED_VALS = 7;  // rho, j_x, j_y, j_z, G, non-finite count, inadmissible count

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The admissible set of a cell state: rho > 0 and b rho < 1 (the van der
// Waals domain, eq. Pvdw), 0 < theta < 1/3 (theta = P/rho; the practical
// stability bound theta < dx^2/(3 dt^2) of Section 5) and theta + u_a^2 < 1
// on every axis (the rest factor 1 - theta - u_a^2 of eq. phi stays
// positive).  Evaluated in FP64 on finite inputs.
template <int D>
__device__ __forceinline__ bool admissible(double rho, double theta, const double *u, double b) {
    bool ok = rho > 0.0 && b * rho < 1.0 && theta > 0.0 && theta < 1.0 / 3.0;
    for (int a = 0; a < D; a++) ok = ok && theta + u[a] * u[a] < 1.0;
    return ok;
}

// per-block partial sums of the RED_VALS values, written by lane k < RED_VALS
// of the block in a fixed order (wavefront shuffles, then LDS)
__device__ __forceinline__ void block_partials(double (&acc)[RED_VALS], double *partials) {
    __shared__ double sh[RED_VALS][RED_BLOCK / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < RED_VALS; k++) {
        double s = wave_sum(acc[k]);
        if (lane == 0) sh[k][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < RED_VALS) {
        double s = 0;
        for (int i = 0; i < RED_BLOCK / 64; i++) s += sh[threadIdx.x][i];
        partials[(long long)blockIdx.x * RED_VALS + threadIdx.x] = s;
    }
}

template <int D, class C>
__global__ void __launch_bounds__(RED_BLOCK) k_reduce_partials(long long N, Fields<C> fl, double b, double *partials) {
    double acc[RED_VALS] = {0, 0, 0, 0, 0, 0, 0};
    for (long long c = blockIdx.x * (long long)RED_BLOCK + threadIdx.x; c < N; c += (long long)gridDim.x * RED_BLOCK) {
        double rho = fl.rho[c];
        double G = fl.G[c];
        double P = fl.P[c];
        bool bad = !isfinite(rho) || !isfinite(G) || !isfinite(P);
        acc[0] += rho;
        double u[3] = {0, 0, 0};
        for (int a = 0; a < D; a++) {
            double j = (double)fl.J[a * N + c] + 0.5 * (double)fl.F[a * N + c];
            acc[1 + a] += j;
            u[a] = fl.u[a * N + c];
            bad = bad || !isfinite(j) || !isfinite(u[a]);
        }
        acc[4] += G;
        acc[5] += bad ? 1.0 : 0.0;
        acc[6] += (!bad && !admissible<D>(rho, P / rho, u, b)) ? 1.0 : 0.0;
    }
    block_partials(acc, partials);
}

// the same counts for the FP64 inputs of lbm_init (rho, u, T given; P from
// eq. Pvdw), columns 5 and 6 of the partials, the others zero
template <int D>
__global__ void __launch_bounds__(RED_BLOCK) k_check_inputs(long long N, Phys<double> ph, const double *rho,
                                                            const double *u, const double *T, double *partials) {
    double acc[RED_VALS] = {0, 0, 0, 0, 0, 0, 0};
    for (long long c = blockIdx.x * (long long)RED_BLOCK + threadIdx.x; c < N; c += (long long)gridDim.x * RED_BLOCK) {
        const double r = rho[c], t = T[c];
        double uu[3] = {0, 0, 0};
        bool bad = !isfinite(r) || !isfinite(t);
        for (int a = 0; a < D; a++) {
            uu[a] = u[a * N + c];
            bad = bad || !isfinite(uu[a]);
        }
        acc[5] += bad ? 1.0 : 0.0;
        if (!bad) {
            const double P = ph.pr ? pr_eos(ph, r, t).P : vdw_pressure(ph, r, t);
            acc[6] += admissible<D>(r, P / r, uu, ph.b) ? 0.0 : 1.0;
        }
    }
    block_partials(acc, partials);
}

__global__ void __launch_bounds__(64) k_reduce_final(int nblocks, const double *partials, double *out) {
    // one wave; lane k < RED_VALS sums column k in block order
    int k = threadIdx.x;
    if (k < RED_VALS) {
        double s = 0;
        for (int b = 0; b < nblocks; b++) s += partials[(long long)b * RED_VALS + k];
        out[k] = s;
    }
}

// population decode / encode between the storage form and FP64
template <int D, class S>
__global__ void __launch_bounds__(BX) k_get_pops(Grid g, RefPops ref, const typename S::T *fi, const typename S::T *gi,
                                                 double *fo, double *go, int pull) {
    using C = typename S::C;
    constexpr int Q = Lattice<D>::Q;
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    long long c = cell_index<D>(g, x, y, z);
    for (int i = 0; i < Q; i++) {
        const long long pi = arrived_index<D>(g, i, x, y, z, pull);
        fo[i * g.N + c] = (double)S::load(fi, pi, (C)ref.f[i]);
        go[i * g.N + c] = (double)S::load(gi, pi, (C)ref.g[i]);
    }
}
template <int D, class S>
__global__ void __launch_bounds__(BX) k_set_pops(Grid g, RefPops ref, const double *fi, const double *gi,
                                                 typename S::T *fo, typename S::T *go) {
    using C = typename S::C;
    constexpr int Q = Lattice<D>::Q;
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    long long c = cell_index<D>(g, x, y, z);
    const long long xy = x + (long long)g.nx * y;
    for (int i = 0; i < Q; i++) {
        fo[pop_index<Q>(g, i, z, xy)] = S::enc((C)fi[i * g.N + c], (C)ref.f[i]);
        go[pop_index<Q>(g, i, z, xy)] = S::enc((C)gi[i * g.N + c], (C)ref.g[i]);
    }
}
template <int D, class C>
__global__ void __launch_bounds__(BX) k_export_moments(Grid g, Fields<C> fl, double *rho, double *u, double *T,
                                                       double *P) {
    int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= g.nx) return;
    long long c = cell_index<D>(g, x, y, z);
    if (rho) rho[c] = fl.rho[c];
    if (u)
        for (int a = 0; a < D; a++) u[a * g.N + c] = fl.u[a * g.N + c];
    if (T) T[c] = fl.T[c];
    if (P) P[c] = fl.P[c];
}

__global__ void k_codec_encode(int kind, const float *x, const float *ref, uint16_t *out, long long n) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float d = x[i] - ref[i];
    out[i] = kind == LBM_STORE_BF16 ? f32_to_bf16_rne(d) : f32_to_f16_rne(d);
}
__global__ void k_codec_decode(int kind, const uint16_t *code, const float *ref, float *out, long long n) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = ref[i] + (kind == LBM_STORE_BF16 ? bf16_to_f32(code[i]) : f16_to_f32(code[i]));
}
// HBM bandwidth probes (the practical ceiling the step's kernels are
// measured against): 16-byte accesses per lane, grid-stride loops, stores
// and loads with the non-temporal hint.  The read probe folds its loads into
// one value that is stored only if it equals an arbitrary constant, so the
// loads cannot be dropped.
__global__ void __launch_bounds__(256) k_probe_read(const u32x4 *__restrict__ src, long long n,
                                                    u32x4 *__restrict__ sink) {
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        acc ^= __builtin_nontemporal_load(&src[i]);
    const unsigned a = acc.x, b = acc.y, c = acc.z, d = acc.w;
    if ((a ^ b ^ c ^ d) == 0x9e3779b9u) sink[0] = acc;
}
__global__ void __launch_bounds__(256) k_probe_write(u32x4 *__restrict__ dst, long long n) {
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const unsigned k = (unsigned)i;
        __builtin_nontemporal_store((u32x4){k, k + 1u, k + 2u, k + 3u}, &dst[i]);
    }
}
__global__ void __launch_bounds__(256) k_probe_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                    long long n) {
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}
}  // namespace lbm

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
static dim3 cell_grid(const lbm_ctx *c) {
    return dim3((unsigned)((c->p.nx + BX - 1) / BX), (unsigned)c->p.ny, (unsigned)c->p.nz);
}

static thread_local char g_last_error[256] = "";

int lbm_note(hipError_t e) {
    if (e == hipSuccess) return LBM_OK;
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", hipGetErrorName(e), hipGetErrorString(e));
    return LBM_EDEVICE;
}

static int hip_status(hipError_t e) { return lbm_note(e); }

static int last_launch() { return hip_status(hipGetLastError()); }

template <class C> static Phys<C> make_phys(const lbm_params &p) {
    Phys<C> ph;
    ph.a = (C)p.a; ph.b = (C)p.b; ph.R = (C)p.R; ph.cv = (C)p.cv;
    ph.mu = (C)p.mu; ph.eta = (C)p.eta; ph.k = (C)p.k; ph.kappa = (C)p.kappa;
    ph.inv_cv = (C)(1.0 / p.cv);
    ph.k_over_mu = (C)(p.k / p.mu);
    ph.eta_over_mu = (C)(p.eta / p.mu);
    ph.sgn_eps = (C)p.upwind_eps;
    ph.sc_cmu = (C)p.sc_cmu;
    ph.sc_ceta = (C)p.sc_ceta;
    ph.sc_ck = (C)p.sc_ck;
    ph.pr = lbm_eos_is_pr(p.eos) ? 1 : 0;
    ph.pr_m = p.pr_m;
    ph.pr_Tc = p.pr_Tc;
    ph.pr_c0 = p.pr_c0;
    ph.pr_c1 = p.pr_c1;
    return ph;
}

// reference populations of the 16-bit forms: rest equilibria at (ref_rho,
// ref_T) (Psi(0) = 1 - theta, Psi(+-1) = theta/2 at u = 0), computed in FP64.
static void make_ref(const lbm_params &p, int D, RefPops &ref) {
    std::memset(&ref, 0, sizeof(ref));
    if (!(p.ref_rho > 0 && p.ref_T > 0)) return;
    double r = p.ref_rho, t = p.ref_T;
    double P = r * p.R * t / (1.0 - p.b * r) - p.a * r * r;
    double th = P / r;
    double e = p.cv * t - p.a * r;
    int Q = D == 2 ? 9 : 27;
    // per axis at u = 0: p(0) = 1 - th, p(+-1) = th/2; q(0) = th - 3 th^2,
    // q(+-1) = 3 th^2 / 2
    for (int i = 0; i < Q; i++) {
        int cc[3] = {cx_of(i), cy_of(i), D == 3 ? cz_of(i) : 0};
        double pa[3], qa[3];
        for (int a = 0; a < D; a++) {
            pa[a] = cc[a] ? 0.5 * th : 1.0 - th;
            qa[a] = cc[a] ? 1.5 * th * th : th - 3.0 * th * th;
        }
        double prod = 1.0, s = 0.0;
        for (int a = 0; a < D; a++) prod *= pa[a];
        for (int b = 0; b < D; b++) {
            double t2 = qa[b];
            for (int a = 0; a < D; a++)
                if (a != b) t2 *= pa[a];
            s += t2;
        }
        double feq = r * prod;
        ref.f[i] = (float)feq;
        ref.g[i] = (float)(feq * (e - 0.5 * D * th) + 0.5 * r * s);
    }
}

// ---------------------------------------------------------------------------
// dispatch over (lattice, storage)
// ---------------------------------------------------------------------------
// tile of the fused step.  FP64 uses a smaller tile to fit the LDS budget;
// the other forms take a wide 64 x 4 tile (fewer x-shifted row fragments per
// plane; measured faster than 32 x 8 for FP32 and, fix-up pass included,
// for BF16).
template <class S, bool MLP>
using TileOf = typename std::conditional<std::is_same<S, StoreF64>::value, Tile<16, 8>, Tile<64, 4>>::type;

template <int D, class S> struct Impl {
    using C = typename S::C;
    using T = typename S::T;
    // the fused step's surrogate form (van der Waals with the network)
    static bool mlp(const lbm_ctx *c) { return std::is_same<C, float>::value && c->p.eos == LBM_EOS_MLP; }

    // complete moments of the current state into the side channel; inbound
    // slots of both buffers start at zero (slots behind a zero-gradient wall
    // are never written afterwards, the fix-up pass adds them as zeros)
    static int fused_prepare(lbm_ctx *c) { return mlp(c) ? fused_prepare_t<true>(c) : fused_prepare_t<false>(c); }
    template <bool M> static int fused_prepare_t(lbm_ctx *c) {
        using TL = TileOf<S, M>;
        if (!c->fused) return LBM_OK;
        for (int s = 0; s < 2; s++) {
            if (hipMemsetAsync(c->Mc[s], 0, c->mc_bytes, c->stream) != hipSuccess ||
                hipMemsetAsync(c->IN[s], 0, c->in_bytes, c->stream) != hipSuccess)
                return lbm_note(hipGetLastError());
        }
        C rs[4];
        ref_sums(c, rs);
        hipLaunchKernelGGL((k_fused_moments<D, S, TL>), cell_grid(c), dim3(BX), 0, c->stream, c->grid, c->ref, rs[0],
                           rs[1], rs[2], rs[3],
                           c->ntx, c->nty, c->nseg, c->nlay, (const T *)c->f[c->cur], (const T *)c->g[c->cur],
                           (C *)c->Mc[c->mcc], c->pulled);
        c->mc_pending = false;
        return last_launch();
    }
    // sums of the reference populations in the compute type as hi + lo
    // pairs {f_hi, f_lo, g_hi, g_lo} (FP64 sums of the stored references)
    static void ref_sums(const lbm_ctx *c, C rs[4]) {
        double sf = 0, sg = 0;
        for (int i = 0; i < c->Q; i++) {
            sf += (double)(C)c->ref.f[i];
            sg += (double)(C)c->ref.g[i];
        }
        rs[0] = (C)sf;
        rs[1] = (C)(sf - (double)rs[0]);
        rs[2] = (C)sg;
        rs[3] = (C)(sg - (double)rs[2]);
    }
    // full tiles and periodic x, y: the instance without wall and
    // partial-tile handling.  With 16-bit storage and the explicit EOS that
    // instance also completes its input moments itself (kfold) and needs z
    // segments of at least 6 planes; shorter ones take the general instance.
    static constexpr bool fold_storage = sizeof(T) == 2;
    template <bool M> static bool fast_instance(const lbm_ctx *c) {
        using TL = TileOf<S, M>;
        const bool fast = c->p.nx % TL::TX == 0 && c->p.ny % TL::TY == 0 && c->p.bc[0] == LBM_BC_PERIODIC &&
                          c->p.bc[1] == LBM_BC_PERIODIC;
        if (!fast || M || !fold_storage || D == 2) return fast;
        return c->p.nz / c->nseg >= 6;
    }
    static bool kfold(const lbm_ctx *c) { return fold_storage && !mlp(c) && c->fused && fast_instance<false>(c); }
    // the fused step proper (kind 0 of step_timed)
    static void fused_main(lbm_ctx *c) { mlp(c) ? fused_main_t<true>(c) : fused_main_t<false>(c); }
    template <bool M> static void fused_main_t(lbm_ctx *c) {
        using TL = TileOf<S, M>;
        FusedArgs<C, T> a;
        a.g = c->grid;
        a.ph = make_phys<C>(c->p);
        a.ref = c->ref;
        a.ntx = c->ntx;
        a.nty = c->nty;
        a.nseg = c->nseg;
        a.nlay = c->nlay;
        a.chunk = c->chunk;
        a.pull = c->pulled;
        {
            C rs[4];
            ref_sums(c, rs);
            a.rsf_hi = rs[0];
            a.rsf_lo = rs[1];
            a.rsg_hi = rs[2];
            a.rsg_lo = rs[3];
        }
        const int nxt = 1 - c->cur;
        a.fi = (const T *)c->f[c->cur];
        a.fo = (T *)c->f[nxt];
        a.Mci = (const C *)c->Mc[c->mcc];
        a.Mco = (C *)c->Mc[1 - c->mcc];
        a.INo = (C *)c->IN[1 - c->mcc];
        a.INi = (const C *)c->IN[c->mcc];
        a.Tin = (const C *)c->Tsur;
        a.Acc = (const unsigned *)c->Acc;
        a.accw = 2 * ((c->p.nx + 63) / 64);
        a.inv_cv_d = 1.0 / (double)(float)c->p.cv;
        const dim3 grid((unsigned)(c->ntx * c->nty * c->nseg));
        const bool fast = fast_instance<M>(c);
        if constexpr (M && std::is_same<C, float>::value) {
            if (fast) hipLaunchKernelGGL((k_fused<D, S, TL, true, true>), grid, dim3(TL::NT), 0, c->stream, a);
            else hipLaunchKernelGGL((k_fused<D, S, TL, true, false>), grid, dim3(TL::NT), 0, c->stream, a);
        } else {
            if (fast) hipLaunchKernelGGL((k_fused<D, S, TL, false, true>), grid, dim3(TL::NT), 0, c->stream, a);
            else hipLaunchKernelGGL((k_fused<D, S, TL, false, false>), grid, dim3(TL::NT), 0, c->stream, a);
        }
        c->cur = nxt;
        c->pulled = 1;
        c->mc_pending = true;
    }
    // the surrogate pass completes the side channel itself (the fix-up's
    // work): the surrogate form on 64 x 4 tiles, every tile at least 2 x 2
    static bool fold(const lbm_ctx *c) {
        return mlp(c) && c->p.nx >= 2 && c->p.ny >= 2 && c->p.nx % 64 != 1 && c->p.ny % 4 != 1;
    }
    // completes the output moments (kind 1 of step_timed) and flips the state;
    // after a folding step only the segment-end planes (the next step adds
    // the perimeter cells' slots on load).  In the surrogate form with the
    // completion in its pass, only the segment-end planes too, and the state
    // stays pending: the pass adds the perimeter cells' slots and writes the
    // complete moments to the other buffer.
    static void fused_fixup(lbm_ctx *c) { mlp(c) ? fused_fixup_t<true>(c) : fused_fixup_t<false>(c); }
    template <bool M> static void fused_fixup_t(lbm_ctx *c) {
        using TL = TileOf<S, M>;
        if (!c->mc_pending) return;
        const int nxt = 1 - c->mcc;
        if (fold(c)) {
            if (D == 3) {
                const long long plane = (long long)c->p.nx * c->p.ny;
                hipLaunchKernelGGL((k_fused_fixup<D, TL, C>), dim3((unsigned)((plane + BX - 1) / BX), 2 * c->nseg),
                                   dim3(BX), 0, c->stream, c->grid, c->ntx, c->nty, c->nseg, 1,
                                   (C *)c->Mc[nxt], (const C *)c->IN[nxt]);
            }
            return;
        }
        const long long per = (long long)c->ntx * c->nty * TL::PMAX;
        if (!kfold(c))
            hipLaunchKernelGGL((k_fused_fixup<D, TL, C>), dim3((unsigned)((per + BX - 1) / BX), c->p.nz), dim3(BX),
                               0, c->stream, c->grid, c->ntx, c->nty, c->nseg, 0, (C *)c->Mc[nxt],
                               (const C *)c->IN[nxt]);
        if (D == 3) {
            const long long plane = (long long)c->p.nx * c->p.ny;
            hipLaunchKernelGGL((k_fused_fixup<D, TL, C>), dim3((unsigned)((plane + BX - 1) / BX), 2 * c->nseg),
                               dim3(BX), 0, c->stream, c->grid, c->ntx, c->nty, c->nseg, 1,
                               (C *)c->Mc[nxt], (const C *)c->IN[nxt]);
        }
        c->mcc = nxt;
        c->mc_pending = false;
    }
    // surrogate form: T of every cell by the network pass (kind 2 of
    // step_timed), ahead of the fused step that reads it
    static void fused_eos(lbm_ctx *c) {
        if constexpr (std::is_same<C, float>::value) {
            if (!mlp(c)) return;
            // 64 x 4 columns per workgroup, marching through the fewest chunks
            // of at most 58 planes, as even as nz allows (longer chunks spread
            // the prologue -- rho region of four planes, two Laplacians, the
            // permuted weights -- over more planes: at 512^3, 32 -> 56 took the
            // pass 2.98 -> 2.88 ms, nine chunks of 57 and 56 instead of nine of
            // 56 and one of 8 2.39 -> 2.36 ms; the end-plane bitmask of the
            // completing pass spans a chunk plus 6 planes, at most 64)
            constexpr int ZCHUNK_MAX = 58;
            static_assert(ZCHUNK_MAX + 6 <= 64, "end-plane bitmask of the surrogate pass");
            const int nchunk = D == 3 ? (c->p.nz + ZCHUNK_MAX - 1) / ZCHUNK_MAX : 1;
            const int zchunk = D == 3 ? (c->p.nz + nchunk - 1) / nchunk : 1;
            const dim3 grid((unsigned)((c->p.nx + 63) / 64), (unsigned)((c->p.ny + 3) / 4),
                            (unsigned)((c->p.nz + zchunk - 1) / zchunk));
            FoldArgs fa{nullptr, nullptr, c->ntx, c->nty, c->nseg};
            if (fold(c) && c->mc_pending) {
                // partial sums and slots of the last fused step in (its
                // segment-end planes completed by the fix-up), complete
                // moments out to the buffer that step read
                fa.IN = (const float *)c->IN[1 - c->mcc];
                fa.Mco = (float *)c->Mc[c->mcc];
                hipLaunchKernelGGL((k_eos_surrogate<D, true>), grid, dim3(256), 0, c->stream, c->grid,
                                   make_phys<float>(c->p), (const float *)c->Mc[1 - c->mcc], (float *)c->Tsur,
                                   c->mlp_params, c->mlp_w2b, c->mlp_norm, (float)c->p.mlp_tol, c->mlp_counters,
                                   zchunk, fa, (unsigned long long *)c->Acc);
                c->mc_pending = false;
            } else {
                hipLaunchKernelGGL((k_eos_surrogate<D, false>), grid, dim3(256), 0, c->stream, c->grid,
                                   make_phys<float>(c->p), (const float *)c->Mc[c->mcc], (float *)c->Tsur,
                                   c->mlp_params, c->mlp_w2b, c->mlp_norm, (float)c->p.mlp_tol, c->mlp_counters,
                                   zchunk, fa, (unsigned long long *)c->Acc);
            }
        }
    }
    static void fused_launch(lbm_ctx *c) {
        fused_eos(c);
        fused_main(c);
        fused_fixup(c);
    }

    // counts of non-finite and inadmissible cells of the inputs (blocking)
    static int check_inputs(lbm_ctx *c, const double *rho, const double *u, const double *Tf) {
        hipLaunchKernelGGL((k_check_inputs<D>), dim3(c->red_blocks), dim3(RED_BLOCK), 0, c->stream,
                           (long long)c->grid.N, make_phys<double>(c->p), rho, u, Tf, c->red_partials);
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, c->stream, c->red_blocks, c->red_partials,
                           c->red_out);
        int rc = last_launch();
        if (rc) return rc;
        double tmp[RED_VALS];
        if (hipMemcpyAsync(tmp, c->red_out, sizeof(tmp), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return lbm_note(hipGetLastError());
        return tmp[5] > 0 ? LBM_ENAN : (tmp[6] > 0 ? LBM_EUNSTABLE : LBM_OK);
    }
    static int init(lbm_ctx *c, const double *rho, const double *u, const double *Tf) {
        int rc0 = check_inputs(c, rho, u, Tf);
        if (rc0) return rc0;
        hipLaunchKernelGGL((k_init<D, S>), cell_grid(c), dim3(BX), 0, c->stream, c->grid, make_phys<double>(c->p), c->ref,
                           rho, u, Tf, (T *)c->f[c->cur], (T *)c->g[c->cur]);
        c->pulled = 0;
        int rc = last_launch();
        return rc ? rc : fused_prepare(c);
    }
    // count: add the Peng-Robinson Newton iterations to the context's
    // counters (the step's passes; read-back passes do not count)
    static int fields_pass(lbm_ctx *c, bool count = false) {
        Fields<C> fl = get_fields<C>(c);
        dim3 gr = cell_grid(c);
        hipLaunchKernelGGL((k_moments<D, S>), gr, dim3(BX), 0, c->stream, c->grid, c->ref, (const T *)c->f[c->cur],
                           (const T *)c->g[c->cur], fl, c->pulled);
        hipLaunchKernelGGL((k_lap<D, C>), gr, dim3(BX), 0, c->stream, c->grid, fl);
        if (lbm_eos_uses_mlp(c->p.eos)) {
            int rc = launch_fields_mlp<D, C>(c, fl, count);
            if (rc) return rc;
        } else {
            hipLaunchKernelGGL((k_fields<D, C>), gr, dim3(BX), 0, c->stream, c->grid, make_phys<C>(c->p), fl,
                               (c->p.eos == LBM_EOS_PR_PREV && c->T_valid) ? 1 : 0,
                               count ? c->mlp_counters + 2 : (unsigned long long *)nullptr);
        }
        c->T_valid = true;
        return last_launch();
    }
    // shock-capturing passes over the fields of the step; returns the filtered
    // (|grad^4 S|, |grad^4 |grad s||) arrays, or nulls when the scheme is off
    static void sc_passes(lbm_ctx *c, const C **fS, const C **fs) {
        *fS = *fs = nullptr;
        if (!c->sc) return;
        Fields<C> fl = get_fields<C>(c);
        dim3 gr = cell_grid(c);
        hipLaunchKernelGGL((k_sc_grad<D, C>), gr, dim3(BX), 0, c->stream, c->grid, make_phys<C>(c->p), fl);
        hipLaunchKernelGGL((k_sc_d4<D, C>), gr, dim3(BX), 0, c->stream, c->grid, fl.sc[0], fl.sc[1], fl.sc[2],
                           fl.sc[3]);
        // filter weights exp(-j^2 / (2 sigma^2)), |j| <= 4, sigma = 1.2, normalised
        ScFilter<C> f;
        double w[2 * SC_RADIUS + 1], ws = 0;
        for (int j = -SC_RADIUS; j <= SC_RADIUS; j++) ws += (w[j + SC_RADIUS] = std::exp(-(double)(j * j) / 2.88));
        for (int j = 0; j <= 2 * SC_RADIUS; j++) f.w[j] = (C)(w[j] / ws);
        int src = 2;
        for (int a = 0; a < D; a++) {
            const int dst = 2 - src;
            hipLaunchKernelGGL((k_sc_filter<D, C>), gr, dim3(BX), 0, c->stream, c->grid, a, f, fl.sc[src],
                               fl.sc[src + 1], fl.sc[dst], fl.sc[dst + 1]);
            src = dst;
        }
        *fS = fl.sc[src];
        *fs = fl.sc[src + 1];
    }
    // collide and stream into buffer nxt (multi-kernel path), then what the
    // wall ghosts emit
    static void collide_launch(lbm_ctx *c, Fields<C> fl, const C *fS, const C *fs, int nxt) {
        Walls w;
        for (int s = 0; s < 2; s++) {
            for (int a = 0; a < 3; a++) w.u[s][a] = c->p.wall_u[s][a];
            w.T[s] = c->p.wall_T[s];
        }
        hipLaunchKernelGGL((k_collide<D, S>), cell_grid(c), dim3(BX), 0, c->stream, c->grid, make_phys<C>(c->p),
                           c->ref, (const T *)c->f[c->cur], (const T *)c->g[c->cur], fl, (T *)c->f[nxt],
                           (T *)c->g[nxt], fS, fs, w, (C *)c->ghost);
        if (c->grid.wallx)
            hipLaunchKernelGGL((k_wall_emit<D, S>), dim3((unsigned)((c->p.ny + 63) / 64), (unsigned)c->p.nz, 2u),
                               dim3(64), 0, c->stream, c->grid, make_phys<C>(c->p), c->ref, w, fl,
                               (const C *)c->ghost, (T *)c->f[nxt], (T *)c->g[nxt]);
    }
    static int step(lbm_ctx *c, int n) {
        Fields<C> fl = get_fields<C>(c);
        dim3 gr = cell_grid(c);
        for (int s = 0; s < n; s++) {
            int rc;
            if (c->fused) {
                fused_launch(c);
                rc = last_launch();
            } else {
                rc = fields_pass(c, true);
                if (rc) return rc;
                const C *fS, *fs;
                sc_passes(c, &fS, &fs);
                int nxt = 1 - c->cur;
                collide_launch(c, fl, fS, fs, nxt);
                rc = last_launch();
                c->cur = nxt;
            }
            if (rc) return rc;
            c->steps_done++;
            if (c->p.check_every > 0 && c->steps_done % c->p.check_every == 0) {
                double tmp[RED_VALS];
                rc = conservation(c, tmp);
                if (rc) return rc;
            }
        }
        return LBM_OK;
    }
    // n steps with events between the launches: host_ms[k] receives the
    // average duration of kernel kind k (moments, laplacian, fields, collide)
    static int step_timed(lbm_ctx *c, int n, double *host_ms) {
        hipEvent_t ev[5];
        for (int k = 0; k < 5; k++)
            if (hipEventCreate(&ev[k]) != hipSuccess) return LBM_EDEVICE;
        if (c->fused) {
            // kinds: 0 k_fused, 1 k_fused_fixup, 2 k_eos_surrogate
            double acc[3] = {0, 0, 0};
            const int kind_of[3] = {2, 0, 1};
            int rc = LBM_OK;
            for (int s = 0; s < n && rc == LBM_OK; s++) {
                (void)hipEventRecord(ev[0], c->stream);
                fused_eos(c);
                (void)hipEventRecord(ev[1], c->stream);
                fused_main(c);
                (void)hipEventRecord(ev[2], c->stream);
                fused_fixup(c);
                (void)hipEventRecord(ev[3], c->stream);
                rc = last_launch();
                for (int k = 0; k < 3 && rc == LBM_OK; k++) {
                    float ms = 0;
                    if (hipEventSynchronize(ev[k + 1]) != hipSuccess ||
                        hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess)
                        rc = LBM_EDEVICE;
                    acc[kind_of[k]] += ms;
                }
            }
            for (int k = 0; k < 5; k++) (void)hipEventDestroy(ev[k]);
            for (int k = 0; k < LBM_NUM_KERNELS; k++) host_ms[k] = (k < 3 && n > 0) ? acc[k] / n : 0.0;
            if (!mlp(c)) host_ms[2] = 0.0;
            return rc;
        }
        double acc[4] = {0, 0, 0, 0};
        Fields<C> fl = get_fields<C>(c);
        dim3 gr = cell_grid(c);
        int rc = LBM_OK;
        for (int s = 0; s < n && rc == LBM_OK; s++) {
            (void)hipEventRecord(ev[0], c->stream);
            hipLaunchKernelGGL((k_moments<D, S>), gr, dim3(BX), 0, c->stream, c->grid, c->ref,
                               (const T *)c->f[c->cur], (const T *)c->g[c->cur], fl, 0);
            (void)hipEventRecord(ev[1], c->stream);
            hipLaunchKernelGGL((k_lap<D, C>), gr, dim3(BX), 0, c->stream, c->grid, fl);
            (void)hipEventRecord(ev[2], c->stream);
            if (lbm_eos_uses_mlp(c->p.eos)) rc = launch_fields_mlp<D, C>(c, fl, true);
            else
                hipLaunchKernelGGL((k_fields<D, C>), gr, dim3(BX), 0, c->stream, c->grid, make_phys<C>(c->p), fl,
                                   (c->p.eos == LBM_EOS_PR_PREV && c->T_valid) ? 1 : 0, c->mlp_counters + 2);
            c->T_valid = true;
            const C *fS, *fs;
            sc_passes(c, &fS, &fs);  // timed with the fields kind
            (void)hipEventRecord(ev[3], c->stream);
            int nxt = 1 - c->cur;
            collide_launch(c, fl, fS, fs, nxt);
            (void)hipEventRecord(ev[4], c->stream);
            if (rc == LBM_OK) rc = last_launch();
            c->cur = nxt;
            if (hipEventSynchronize(ev[4]) != hipSuccess) rc = LBM_EDEVICE;
            for (int k = 0; k < 4 && rc == LBM_OK; k++) {
                float ms = 0;
                if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) rc = LBM_EDEVICE;
                acc[k] += ms;
            }
        }
        for (int k = 0; k < 5; k++) (void)hipEventDestroy(ev[k]);
        for (int k = 0; k < 4; k++) host_ms[k] = n > 0 ? acc[k] / n : 0.0;
        return rc;
    }
    static int moments(lbm_ctx *c, double *rho, double *u, double *Tf, double *P) {
        int rc = fields_pass(c);
        if (rc) return rc;
        hipLaunchKernelGGL((k_export_moments<D, C>), cell_grid(c), dim3(BX), 0, c->stream, c->grid, get_fields<C>(c),
                           rho, u, Tf, P);
        return last_launch();
    }
    static int get_pops(lbm_ctx *c, double *f, double *g) {
        hipLaunchKernelGGL((k_get_pops<D, S>), cell_grid(c), dim3(BX), 0, c->stream, c->grid, c->ref,
                           (const T *)c->f[c->cur], (const T *)c->g[c->cur], f, g, c->pulled);
        return last_launch();
    }
    static int set_pops(lbm_ctx *c, const double *f, const double *g) {
        hipLaunchKernelGGL((k_set_pops<D, S>), cell_grid(c), dim3(BX), 0, c->stream, c->grid, c->ref, f, g,
                           (T *)c->f[c->cur], (T *)c->g[c->cur]);
        c->pulled = 0;
        int rc = last_launch();
        return rc ? rc : fused_prepare(c);
    }
    static void tiles(lbm_ctx *c) {
        mlp(c) ? tiles_t<true>(c) : tiles_t<false>(c);
        c->folded = fold(c);
    }
    template <bool M> static void tiles_t(lbm_ctx *c) {
        using TL = TileOf<S, M>;
        c->ntx = (c->p.nx + TL::TX - 1) / TL::TX;
        c->nty = (c->p.ny + TL::TY - 1) / TL::TY;
        const long long ntiles = (long long)c->ntx * c->nty;
        if (D == 2) {
            c->nseg = 1;
        } else if (c->p.zsegments > 0) {
            c->nseg = c->p.zsegments;
        } else {
            // segments of at least 16 planes; the count minimises the
            // workgroup rounds times the planes per segment (no half-empty
            // last round).  Among equal costs: segments of at least 64
            // planes where there are such (the prologue, about 8 planes of
            // loads, stays small), the first count giving 8 workgroups per
            // resident slot, else the longest of them -- a march of one or
            // two rounds ends on its slowest workgroups (512^3, 16-bit: one
            // segment, two rounds, 9.6 ms; four segments 9.0 ms); without
            // such segments the first count reaching 1024 workgroups.
            // Resident workgroups: compute units x the fused kernel's
            // occupancy (the instance the step launches); if the device
            // cannot be queried, the first count giving 1024 workgroups.
            const int smax = std::max(1, c->p.nz / 16);
            int dev = 0, ncu = 0, nb = 0;
            const bool known =
                hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &nb, k_fused<D, S, TL, M && std::is_same<C, float>::value, false>, TL::NT, 0) ==
                    hipSuccess &&
                ncu > 0 && nb > 0;
            if (!known) {
                (void)hipGetLastError();
                c->nseg = std::max(1, std::min((int)((1024 + ntiles - 1) / ntiles), smax));
            } else {
                const long long res = (long long)ncu * nb;
                const int nz = c->p.nz;
                auto cost = [&](int s) { return ((ntiles * s + res - 1) / res) * ((nz + s - 1) / s); };
                long long best_cost = -1;
                for (int s = 1; s <= smax; s++) best_cost = best_cost < 0 ? cost(s) : std::min(best_cost, cost(s));
                int best = -1;
                for (int s = 1; s <= smax && nz / s >= 64; s++) {
                    if (cost(s) != best_cost) continue;
                    best = s;
                    if (ntiles * s >= 8 * res) break;
                }
                if (best < 0) {
                    for (int s = 1; s <= smax; s++) {
                        if (cost(s) != best_cost) continue;
                        best = s;
                        if (ntiles * s >= 1024) break;
                    }
                }
                c->nseg = best;
            }
        }
        c->nlay = D == 3 ? c->p.nz + 2 * c->nseg : 1;
        const long long total = ntiles * c->nseg;
        c->chunk = total % 8 == 0 ? (int)(total / 8) : 0;
        c->mc_bytes = sizeof(C) * 5 * (size_t)c->nlay * c->p.nx * c->p.ny;
        c->in_bytes = sizeof(C) * (size_t)ntiles * c->nlay * 5 * TL::NR;
    }
    static int conservation(lbm_ctx *c, double *host_out) {
        int rc = fields_pass(c);
        if (rc) return rc;
        hipLaunchKernelGGL((k_reduce_partials<D, C>), dim3(c->red_blocks), dim3(RED_BLOCK), 0, c->stream,
                           (long long)c->grid.N, get_fields<C>(c), c->p.b, c->red_partials);
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, c->stream, c->red_blocks, c->red_partials,
                           c->red_out);
        rc = last_launch();
        if (rc) return rc;
        double tmp[RED_VALS];
        if (hipMemcpyAsync(tmp, c->red_out, sizeof(tmp), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return LBM_EDEVICE;
        host_out[0] = tmp[0];
        for (int a = 0; a < D; a++) host_out[1 + a] = tmp[1 + a];
        host_out[D + 1] = tmp[4];
        host_out[D + 2] = tmp[5];
        host_out[D + 3] = tmp[6];
        return tmp[5] > 0 ? LBM_ENAN : (tmp[6] > 0 ? LBM_EUNSTABLE : LBM_OK);
    }
};

#define DISPATCH(ctx, CALL)                                                                    \
    do {                                                                                       \
        const int st_ = (ctx)->p.storage;                                                      \
        if ((ctx)->D == 2) {                                                                   \
            if (st_ == LBM_STORE_F64) return Impl<2, StoreF64>::CALL;                          \
            if (st_ == LBM_STORE_F32) return Impl<2, StoreF32>::CALL;                          \
            if (st_ == LBM_STORE_BF16) return Impl<2, StoreBF16>::CALL;                        \
            return Impl<2, StoreF16>::CALL;                                                    \
        }                                                                                      \
        if (st_ == LBM_STORE_F64) return Impl<3, StoreF64>::CALL;                              \
        if (st_ == LBM_STORE_F32) return Impl<3, StoreF32>::CALL;                              \
        if (st_ == LBM_STORE_BF16) return Impl<3, StoreBF16>::CALL;                            \
        return Impl<3, StoreF16>::CALL;                                                        \
    } while (0)

#define DISPATCH_VOID(ctx, CALL)                                                               \
    do {                                                                                       \
        const int st_ = (ctx)->p.storage;                                                      \
        if ((ctx)->D == 2) {                                                                   \
            if (st_ == LBM_STORE_F64) Impl<2, StoreF64>::CALL;                                 \
            else if (st_ == LBM_STORE_F32) Impl<2, StoreF32>::CALL;                            \
            else if (st_ == LBM_STORE_BF16) Impl<2, StoreBF16>::CALL;                          \
            else Impl<2, StoreF16>::CALL;                                                      \
        } else {                                                                               \
            if (st_ == LBM_STORE_F64) Impl<3, StoreF64>::CALL;                                 \
            else if (st_ == LBM_STORE_F32) Impl<3, StoreF32>::CALL;                            \
            else if (st_ == LBM_STORE_BF16) Impl<3, StoreBF16>::CALL;                          \
            else Impl<3, StoreF16>::CALL;                                                      \
        }                                                                                      \
    } while (0)

// ---------------------------------------------------------------------------
// exported entry points
// ---------------------------------------------------------------------------
extern "C" {

const char *lbm_strerror(int s) {
    switch (s) {
        case LBM_OK: return "ok";
        case LBM_EINVAL: return "invalid argument";
        case LBM_ENOMEM: return "device allocation failed";
        case LBM_EDEVICE: return "HIP runtime or kernel launch error";
        case LBM_EUNSTABLE: return "state left the admissible set";
        case LBM_ENAN: return "non-finite value in the state";
        case LBM_ESTATE: return "call out of order";
        default: return "unknown status";
    }
}

static int validate(const lbm_params *p) {
    if (!p) return LBM_EINVAL;
    if (p->lattice != 2 && p->lattice != 3) return LBM_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return LBM_EINVAL;
    if (p->lattice == 2 && p->nz != 1) return LBM_EINVAL;
    if (p->ny > 65535 || p->nz > 65535) return LBM_EINVAL;
    for (int a = 0; a < 3; a++)
        if (p->bc[a] != LBM_BC_PERIODIC && p->bc[a] != LBM_BC_ZEROGRAD && !(a == 0 && p->bc[a] == LBM_BC_WALL))
            return LBM_EINVAL;
    if (p->bc[0] == LBM_BC_WALL) {
        if (p->bc[1] != LBM_BC_PERIODIC || p->bc[2] != LBM_BC_PERIODIC) return LBM_EINVAL;
        for (int s = 0; s < 2; s++)
            if (!(p->wall_T[s] > 0) || !std::isfinite(p->wall_u[s][0]) || !std::isfinite(p->wall_u[s][1]) ||
                !std::isfinite(p->wall_u[s][2]))
                return LBM_EINVAL;
    }
    if (p->storage < LBM_STORE_F64 || p->storage > LBM_STORE_F16) return LBM_EINVAL;
    if (p->eos < LBM_EOS_VDW || p->eos > LBM_EOS_PR_MLP) return LBM_EINVAL;
    if (lbm_eos_uses_mlp(p->eos) && p->storage == LBM_STORE_F64) return LBM_EINVAL;
    if (lbm_eos_is_pr(p->eos) && !(p->pr_Tc > 0 && p->pr_c0 > 0 && p->pr_c1 >= 0 && std::isfinite(p->pr_m) &&
                                   p->b > 0 && p->a >= 0))
        return LBM_EINVAL;
    if (!(p->cv > 0) || !(p->mu > 0) || !(p->R > 0)) return LBM_EINVAL;
    if (!(p->upwind_eps >= 0)) return LBM_EINVAL;
    if (p->zsegments < 0 || p->zsegments > p->nz) return LBM_EINVAL;
    if (p->check_every < 0) return LBM_EINVAL;
    if (!(p->sc_cmu >= 0 && p->sc_ceta >= 0 && p->sc_ck >= 0) || !std::isfinite(p->sc_cmu) ||
        !std::isfinite(p->sc_ceta) || !std::isfinite(p->sc_ck))
        return LBM_EINVAL;
    if ((long long)p->nx * p->ny > (1LL << 30)) return LBM_EINVAL;
    if ((p->storage == LBM_STORE_BF16 || p->storage == LBM_STORE_F16) && !(p->ref_rho > 0 && p->ref_T > 0))
        return LBM_EINVAL;
    if (!(p->ref_rho >= 0 && p->ref_T >= 0)) return LBM_EINVAL;
    return LBM_OK;
}

int lbm_create(const lbm_params *params, lbm_ctx **out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    int rc = validate(params);
    if (rc) return rc;
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_ENOMEM;
    c->p = *params;
    c->D = params->lattice;
    c->Q = c->D == 2 ? 9 : 27;
    c->stream = (hipStream_t)params->stream;
    c->grid.nx = params->nx; c->grid.ny = params->ny; c->grid.nz = params->nz;
    c->grid.clampx = params->bc[0] != LBM_BC_PERIODIC; c->grid.clampy = params->bc[1]; c->grid.clampz = params->bc[2];
    c->grid.wallx = params->bc[0] == LBM_BC_WALL;
    c->grid.N = (long long)params->nx * params->ny * params->nz;
    const long long N = c->grid.N;
    int sb = params->storage == LBM_STORE_F64 ? 8 : (params->storage == LBM_STORE_F32 ? 4 : 2);
    c->store_bytes = sb;
    int cb = params->storage == LBM_STORE_F64 ? 8 : 4;
    make_ref(*params, c->D, c->ref);
    size_t pop_bytes = (size_t)c->Q * N * sb;
    // field arrays: rho, J[D], G, lap, u[D], F[D], Lam[D], T, P, h, cs2, and
    // the four shock-capturing work arrays when that scheme is on
    c->sc = params->sc_cmu > 0 || params->sc_ceta > 0 || params->sc_ck > 0;
    size_t nfield = (size_t)(8 + 4 * c->D + (c->sc ? 4 : 0));
    size_t field_bytes = nfield * N * cb;
    // the single-pass step covers periodic z (and every D = 2 lattice)
    // with the van der Waals equation of state, without shock capturing
    c->fused = (c->D == 2 || params->bc[2] == LBM_BC_PERIODIC) && !c->sc && !lbm_eos_is_pr(params->eos) &&
               params->bc[0] != LBM_BC_WALL;
    if (c->fused) {
        auto tiles = [&]() { DISPATCH_VOID(c, tiles(c)); };
        tiles();
        // its buffer resources (one plane of populations, one side-channel
        // layer, one layer of inbound slots) must stay below 2^31 bytes;
        // larger planes take the multi-kernel path
        const long long plane = (long long)params->nx * params->ny, lim = 1LL << 31;
        if (2LL * c->Q * plane * sb >= lim || 5 * plane * cb >= lim || (long long)(c->in_bytes / c->nlay) >= lim)
            c->fused = false;
    }
    if (!c->fused) c->folded = false;
    // The large buffers come from one allocation, carved at 2 MiB boundaries:
    // the population sets (one buffer per ping-pong slot holds both sets, f_i
    // and g_i side by side; the g pointer is the f buffer offset by one
    // element), the field arrays, the wall ghosts, and the fused step's side
    // channel, inbound slots, surrogate temperatures and their acceptance bits.
    struct Part {
        void **dst;
        size_t bytes;
    };
    const bool mlpT = c->fused && params->eos == LBM_EOS_MLP;
    const Part parts[] = {{&c->f[0], 2 * pop_bytes},
                          {&c->f[1], 2 * pop_bytes},
                          {&c->work, field_bytes},
                          {&c->ghost, c->grid.wallx ? (size_t)2 * params->ny * params->nz * c->Q * cb : 0},
                          {&c->Mc[0], c->fused ? c->mc_bytes : 0},
                          {&c->Mc[1], c->fused ? c->mc_bytes : 0},
                          {&c->IN[0], c->fused ? c->in_bytes : 0},
                          {&c->IN[1], c->fused ? c->in_bytes : 0},
                          {&c->Tsur, mlpT ? sizeof(float) * (size_t)N : 0},
                          {&c->Acc, mlpT ? 8 * (size_t)((params->nx + 63) / 64) * params->ny * params->nz : 0}};
    constexpr size_t ALIGN = (size_t)1 << 21;
    size_t total = 0;
    for (const Part &pt : parts) total += (pt.bytes + ALIGN - 1) / ALIGN * ALIGN;
    c->red_blocks = 1024;
    bool ok = hipMalloc(&c->block, total) == hipSuccess &&
              hipMalloc((void **)&c->red_partials, sizeof(double) * RED_VALS * c->red_blocks) == hipSuccess &&
              hipMalloc((void **)&c->red_out, sizeof(double) * RED_VALS) == hipSuccess &&
              hipMalloc((void **)&c->mlp_counters, sizeof(unsigned long long) * 4) == hipSuccess &&
              hipMalloc((void **)&c->mlp_params, sizeof(float) * (LBM_MLP_NPARAMS + 64)) == hipSuccess &&
              hipMalloc((void **)&c->mlp_norm, sizeof(float) * 16) == hipSuccess &&
              hipMalloc((void **)&c->mlp_w2b, sizeof(uint16_t) * 64 * 64) == hipSuccess;
    if (!ok) {
        lbm_note(hipGetLastError());
        lbm_destroy(c);
        return LBM_ENOMEM;
    }
    {
        char *q = (char *)c->block;
        for (const Part &pt : parts) {
            *pt.dst = pt.bytes ? q : nullptr;
            q += (pt.bytes + ALIGN - 1) / ALIGN * ALIGN;
        }
        for (int k = 0; k < 2; k++) c->g[k] = (char *)c->f[k] + sb;
    }
    (void)hipMemsetAsync(c->mlp_counters, 0, sizeof(unsigned long long) * 4, c->stream);
    c->cur = 0;
    c->mcc = 0;
    c->mc_pending = false;
    c->initialized = false;
    c->mlp_ready = false;
    *out = c;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    // errors here have nowhere to go (the call returns nothing); the context
    // is released regardless
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    // the large buffers are carved from c->block
    void *ptrs[] = {c->block, c->red_partials, c->red_out, c->mlp_counters, c->mlp_params, c->mlp_norm, c->mlp_w2b};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete c;
}

static int init_dispatch(lbm_ctx *c, const double *rho, const double *u, const double *Tf) {
    DISPATCH(c, init(c, rho, u, Tf));
}

int lbm_init(lbm_ctx *c, const double *rho, const double *u, const double *Tf) {
    if (!c || !rho || !u || !Tf) return LBM_EINVAL;
    c->cur = 0;
    c->mcc = 0;
    c->mc_pending = false;
    c->initialized = false;
    const int rc = init_dispatch(c, rho, u, Tf);
    c->initialized = rc == LBM_OK;
    c->steps_done = 0;
    c->T_valid = false;
    return rc;
}

int lbm_step(lbm_ctx *c, int n) {
    if (!c) return LBM_EINVAL;
    if (!c->initialized) return LBM_ESTATE;
    if (n < 0) return LBM_EINVAL;
    if (lbm_eos_uses_mlp(c->p.eos) && !c->mlp_ready) return LBM_ESTATE;
    DISPATCH(c, step(c, n));
}

int lbm_moments(lbm_ctx *c, double *rho, double *u, double *Tf, double *P) {
    if (!c) return LBM_EINVAL;
    if (!c->initialized) return LBM_ESTATE;
    if (lbm_eos_uses_mlp(c->p.eos) && !c->mlp_ready) return LBM_ESTATE;
    DISPATCH(c, moments(c, rho, u, Tf, P));
}

int lbm_get_populations(lbm_ctx *c, double *f, double *g) {
    if (!c || !f || !g) return LBM_EINVAL;
    if (!c->initialized) return LBM_ESTATE;
    DISPATCH(c, get_pops(c, f, g));
}

int lbm_set_populations(lbm_ctx *c, const double *f, const double *g) {
    if (!c || !f || !g) return LBM_EINVAL;
    c->initialized = true;
    c->steps_done = 0;
    c->T_valid = false;
    DISPATCH(c, set_pops(c, f, g));
}

int lbm_conservation(lbm_ctx *c, double *host_out) {
    if (!c || !host_out) return LBM_EINVAL;
    if (!c->initialized) return LBM_ESTATE;
    if (lbm_eos_uses_mlp(c->p.eos) && !c->mlp_ready) return LBM_ESTATE;
    DISPATCH(c, conservation(c, host_out));
}

int lbm_synchronize(lbm_ctx *c) {
    if (!c) return LBM_EINVAL;
    return hip_status(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
}

int lbm_step_timed(lbm_ctx *c, int n, double *host_ms, int nslots) {
    if (!c || !host_ms || n < 0) return LBM_EINVAL;
    if (!c->initialized) return LBM_ESTATE;
    if (lbm_eos_uses_mlp(c->p.eos) && !c->mlp_ready) return LBM_ESTATE;
    if (nslots < LBM_NUM_KERNELS) return LBM_EINVAL;
    DISPATCH(c, step_timed(c, n, host_ms));
}

const char *lbm_last_error(void) { return g_last_error; }

const char *lbm_kernel_name(const lbm_ctx *c, int k) {
    static const char *names[LBM_NUM_KERNELS] = {"k_moments", "k_lap", "k_fields", "k_collide"};
    if (c && c->fused)  // folded: the surrogate pass does the fix-up's work but on the segment-end planes
        return k == 0 ? "k_fused"
                      : (k == 1 ? (c->folded && c->p.lattice == 2 ? "" : "k_fused_fixup")
                                : (k == 2 && c->p.eos == LBM_EOS_MLP ? "k_eos_surrogate" : ""));
    return k >= 0 && k < LBM_NUM_KERNELS ? names[k] : "";
}

int lbm_is_fused(const lbm_ctx *c) { return c && c->fused ? 1 : 0; }

double lbm_bytes_per_cell(const lbm_ctx *c) {
    if (!c) return 0.0;
    return 2.0 * 2.0 * c->Q * c->store_bytes;
}

int lbm_hbm_probe(int kind, const void *src, void *dst, int64_t bytes, int blocks_per_cu, int iters, void *stream,
                  double *host_ms) {
    if (kind < 0 || kind > 2 || bytes <= 0 || bytes % 16 || blocks_per_cu < 1 || blocks_per_cu > 64 || iters < 1 ||
        !host_ms || !dst || (kind != 1 && !src))
        return LBM_EINVAL;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        return lbm_note(hipGetLastError());
    hipStream_t s = (hipStream_t)stream;
    const long long n = bytes / 16;
    const dim3 grid((unsigned)(ncu * blocks_per_cu));
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return lbm_note(hipGetLastError());
    auto launch = [&]() {
        if (kind == 0)
            hipLaunchKernelGGL(k_probe_read, grid, dim3(256), 0, s, (const u32x4 *)src, n, (u32x4 *)dst);
        else if (kind == 1)
            hipLaunchKernelGGL(k_probe_write, grid, dim3(256), 0, s, (u32x4 *)dst, n);
        else
            hipLaunchKernelGGL(k_probe_copy, grid, dim3(256), 0, s, (const u32x4 *)src, (u32x4 *)dst, n);
    };
    launch();  // warm-up
    (void)hipEventRecord(e0, s);
    for (int k = 0; k < iters; k++) launch();
    (void)hipEventRecord(e1, s);
    int rc = last_launch();
    float ms = 0;
    if (rc == LBM_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = lbm_note(hipGetLastError());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *host_ms = (double)ms / iters;
    return rc;
}

int lbm_codec_encode(int kind, const float *x, const float *ref, uint16_t *out, int64_t n, void *stream) {
    if ((kind != LBM_STORE_BF16 && kind != LBM_STORE_F16) || n < 0) return LBM_EINVAL;
    if (n == 0) return LBM_OK;
    if (!x || !ref || !out) return LBM_EINVAL;
    hipLaunchKernelGGL(k_codec_encode, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, kind, x,
                       ref, out, (long long)n);
    return last_launch();
}

int lbm_codec_decode(int kind, const uint16_t *code, const float *ref, float *out, int64_t n, void *stream) {
    if ((kind != LBM_STORE_BF16 && kind != LBM_STORE_F16) || n < 0) return LBM_EINVAL;
    if (n == 0) return LBM_OK;
    if (!code || !ref || !out) return LBM_EINVAL;
    hipLaunchKernelGGL(k_codec_decode, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, kind,
                       code, ref, out, (long long)n);
    return last_launch();
}

}  // extern "C"
