// Library-private definitions shared by the host translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm.h"
#include "lbm_fused.hpp"

struct lbm_ctx {
    lbm_params p;
    lbm::Grid grid;
    int D, Q, store_bytes;
    void *block = nullptr;             // one allocation holding the large buffers below
    void *f[2] = {nullptr, nullptr};  // population state buffers (ping-pong), f_i and g_i side by side
    void *g[2] = {nullptr, nullptr};  // f[k] + one element (not separately allocated)
    int cur = 0;                      // index of the buffer holding the state
    int pulled = 0;                   // 1: the state is the post-collision set (read from x - c_i)
    void *work = nullptr;             // per-cell field arrays
    lbm::RefPops ref;
    hipStream_t stream = nullptr;
    bool initialized = false;
    bool sc = false;                  // shock-capturing numerical transport on
    void *ghost = nullptr;            // LBM_BC_WALL: populations leaving through the walls [2][ny nz][Q]
    long long steps_done = 0;         // steps since the last init / set_populations (check interval)
    bool T_valid = false;             // the field array T holds the current state's temperature
    bool mlp_ready = false;
    int red_blocks = 0;
    double *red_partials = nullptr;
    double *red_out = nullptr;
    unsigned long long *mlp_counters = nullptr;  // [0] fallbacks, [1] evaluations, [2] Newton iterations, [3] cells
    float *mlp_params = nullptr;                 // 4547 FP32 + BF16 copy of W2
    float *mlp_norm = nullptr;
    uint16_t *mlp_w2b = nullptr;      // BF16 copy of the hidden 64x64 weights
    uint16_t mlp_w2b_host[64 * 64];
    // single-pass fused step: moment side channel of the current state
    bool fused = false;
    void *Mc[2] = {nullptr, nullptr};  // [nlay][5][ny][nx]
    void *Tsur = nullptr;              // surrogate form: the network's T of every cell for the fused step
    void *Acc = nullptr;               // and whether it passed the residual check: bits [z][y][x / 64]
    void *IN[2] = {nullptr, nullptr};  // [nlay][tiles][5][slots]
    // side channel state: Mc[mcc] holds the complete moments the next fused
    // step reads; mc_pending: the last fused step's partial sums in
    // Mc[1 - mcc] / IN[1 - mcc] still await completion (by the surrogate pass
    // when it does the fix-up's work)
    int mcc = 0;
    bool mc_pending = false;
    bool folded = false;  // the surrogate pass completes the side channel (the fix-up only its segment-end planes)
    size_t mc_bytes = 0, in_bytes = 0;
    int ntx = 0, nty = 0, nseg = 1, nlay = 0, chunk = 0;
};

// carve the field arrays out of the work buffer
template <class C> static inline lbm::Fields<C> get_fields(lbm_ctx *c) {
    const long long N = c->grid.N;
    const int D = c->D;
    C *w = (C *)c->work;
    lbm::Fields<C> fl;
    fl.rho = w; w += N;
    fl.J = w; w += D * N;
    fl.G = w; w += N;
    fl.lap = w; w += N;
    fl.u = w; w += D * N;
    fl.F = w; w += D * N;
    fl.Lam = w; w += D * N;
    fl.T = w; w += N;
    fl.P = w; w += N;
    fl.h = w; w += N;
    fl.cs2 = w; w += N;
    for (int k = 0; k < 4; k++) {
        fl.sc[k] = c->sc ? w : nullptr;
        if (c->sc) w += N;
    }
    return fl;
}

// Record a failed HIP call's message for lbm_last_error(); returns the status.
int lbm_note(hipError_t e);

// surrogate-EOS variant of the per-cell fields pass (defined with the MLP
// code); count: add Newton iterations to the context's counters
template <int D, class C> int launch_fields_mlp(lbm_ctx *c, lbm::Fields<C> fl, bool count);

// equation-of-state modes
inline bool lbm_eos_is_pr(int eos) { return eos == LBM_EOS_PR || eos == LBM_EOS_PR_PREV || eos == LBM_EOS_PR_MLP; }
inline bool lbm_eos_uses_mlp(int eos) { return eos == LBM_EOS_MLP || eos == LBM_EOS_PR_MLP; }
