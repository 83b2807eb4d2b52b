/*
 * lbm.h -- C ABI of the MI355X (gfx950) fused stream-collide step of the
 * non-ideal compressible double-distribution lattice Boltzmann method of
 * Hosseini, Feinberg & Karlin (arXiv 2510.14712).
 *
 * The calls follow the paper's statement of the problem (Section 3.2 and the
 * flowchart closing it): initialise {f_i, g_i} = {f_i^eq, g_i^eq} from
 * (rho, u, T); iterate "moments -> Korteweg force -> u, E, T, P, Phi, q^c ->
 * attractors -> collide and stream"; read back rho, u, T, P.
 *
 * Conventions shared by every entry point
 *   - Lattice units: dx = dt = 1, lattice speed 1, lattice sound speed^2 = 1/3,
 *     quasi-equilibrium relaxation time lambda = dt (Section 3.2).
 *   - D = 2 uses D2Q9, D = 3 uses D3Q27 (eq. D3Q27c).  Velocity index
 *       i = (c_x + 1) + 3 (c_y + 1) [+ 9 (c_z + 1)],  c_a in {-1, 0, 1}.
 *   - Cell index idx = x + nx (y + ny z), x fastest; nz = 1 when D = 2.
 *   - Fields are FP64 structure-of-arrays: scalar[N], vector[a * N + idx],
 *     populations[i * N + idx], N = nx ny nz.
 *   - Per axis boundary: LBM_BC_PERIODIC, or LBM_BC_ZEROGRAD (populations
 *     entering from outside are the boundary cell's own post-collision
 *     values; finite-difference stencils clamp to the domain).
 *   - Pointers named dev_* are device pointers on the context's device
 *     (e.g. torch.cuda tensors' data_ptr()); they are caller-owned and only
 *     accessed during the call (asynchronously on the context's stream for
 *     calls documented as asynchronous).  Host pointers are named host_*.
 *   - Every function returns LBM_OK (0) or a negative status; no exception
 *     or abort crosses the ABI.  lbm_strerror() names a status.
 *   - A context is not thread-safe; use one context per stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define LBM_OK 0
#define LBM_EINVAL (-1)     /* invalid argument or parameter combination */
#define LBM_ENOMEM (-2)     /* device allocation failed */
#define LBM_EDEVICE (-3)    /* a HIP call or kernel launch failed */
#define LBM_EUNSTABLE (-4)  /* a cell outside the admissible set: rho <= 0,
                               b rho >= 1, theta = P/rho <= 0, theta >= 1/3
                               (the practical stability bound of Section 5,
                               theta < dx^2 / (3 dt^2)) or theta + u_a^2 >= 1
                               on some axis (the rest factor 1 - theta - u_a^2
                               of eq. phi turns negative) */
#define LBM_ENAN (-5)       /* a non-finite value was found */
#define LBM_ESTATE (-6)     /* call out of order (e.g. step before init) */

/* ---- enumerations ------------------------------------------------------ */
#define LBM_BC_PERIODIC 0
#define LBM_BC_ZEROGRAD 1
/* Walls at x = -1 and x = nx (x axis only, y and z periodic): diffuse
 * reflection -- each ghost cell beyond a wall absorbs the populations that
 * leave the domain into it and re-emits the equilibria of the wall state
 * (wall_u, wall_T, and the boundary cell's density for the thermodynamics),
 * scaled to the absorbed mass, so no mass crosses the wall; central
 * differences of u, T, h, Lambda at a boundary cell take the ghost's values,
 * those of rho stay zero-gradient.  The wall treatment of the paper's thermal
 * Couette flow (Section 4.1) is not stated; this is the reading taken.
 * Takes the multi-kernel path. */
#define LBM_BC_WALL 2

/* population storage; arithmetic is FP64 for LBM_STORE_F64 and FP32 for the
 * others.  The two 16-bit forms store f_i - f_i^ref (and g_i - g_i^ref) with
 * round-to-nearest-even, where the reference is the rest equilibrium at
 * (ref_rho, ref_T): f^ref = f^eq(ref_rho, 0, theta_ref), g^ref likewise. */
#define LBM_STORE_F64 0
#define LBM_STORE_F32 1
#define LBM_STORE_BF16 2
#define LBM_STORE_F16 3

/* equation-of-state evaluation inside the step */
#define LBM_EOS_VDW 0       /* explicit van der Waals caloric inversion, eq. lbm_temp */
#define LBM_EOS_MLP 1       /* learned surrogate (rho, e) -> (T, P, c_s^2) with a
                               per-cell residual check and exact Newton fallback */
/* Peng-Robinson (the paper's example of an equation of state whose caloric
 * relation needs an iterative inversion, Section 3.2 after eq. lbm_temp):
 *   P = rho R T / (1 - b rho) - a alpha(T) rho^2 / (1 + 2 b rho - b^2 rho^2),
 *   alpha(T) = (1 + m (1 - sqrt(T / Tc)))^2,
 *   e = c0 T + c1 T^2 / 2 - a (1 + m)(1 + m (1 - sqrt(T / Tc))) L(rho),
 *   L = ln[(1 + (1 + sqrt2) b rho) / (1 + (1 - sqrt2) b rho)] / (2 sqrt2 b),
 * with a, b, R of lbm_params and m, Tc, c0, c1 its pr_* fields (cv unused);
 * T recovered per cell by FP64 Newton iterations to convergence.  These modes
 * take the multi-kernel path. */
#define LBM_EOS_PR 2        /* Newton from the dilute estimate e / c0 */
#define LBM_EOS_PR_PREV 3   /* Newton from the cell's temperature of the previous step */
#define LBM_EOS_PR_MLP 4    /* the surrogate's T, accepted when its caloric residual
                               |e(rho, T_hat) - e| / (c_v T_hat) <= mlp_tol, else
                               Newton from T_hat (not with FP64 storage) */

/* ---- parameters --------------------------------------------------------- */
typedef struct {
    int lattice;            /* 2 (D2Q9) or 3 (D3Q27) */
    int nx, ny, nz;         /* lattice size, nz = 1 for lattice 2 */
    int bc[3];              /* per-axis LBM_BC_* */
    double a, b, R, cv;     /* van der Waals constants (eq. Pvdw) and c_v */
    double mu, eta, k;      /* shear and bulk viscosity, thermal conductivity */
    double kappa;           /* capillarity coefficient (eq. FK) */
    int storage;            /* LBM_STORE_* */
    int eos;                /* LBM_EOS_* */
    double mlp_tol;         /* surrogate acceptance threshold on
                               |e(rho, T_hat) - e| / (c_v T_hat) */
    double ref_rho, ref_T;  /* reference state (rest equilibria at ref_rho,
                               ref_T): required by the 16-bit storage forms,
                               which store deviations from it; optional (0 =
                               none) for FP32/FP64, where it is the origin of
                               the moment sums (accuracy only) */
    void *stream;           /* hipStream_t for all asynchronous work; NULL =
                               the null stream */
    double upwind_eps;      /* |u_a| <= upwind_eps takes the central average in
                               the upwind-biased derivative of Lambda_a (the
                               tie sgn(0) = 0 widened to a round-off dead zone) */
    int zsegments;          /* z segments of the single-pass step (lattice 3,
                               periodic z): 0 = automatic, else 1..nz; the
                               result does not depend on it beyond round-off
                               of the moment sums' order */
    int check_every;        /* > 0: lbm_step checks the state every
                               check_every steps (non-finite cells, then the
                               admissible set of LBM_EUNSTABLE) and returns at
                               the first failing check; 0: no checks */
    double pr_m, pr_Tc, pr_c0, pr_c1; /* Peng-Robinson modes: alpha(T) slope m,
                               critical temperature, ideal-gas heat capacity
                               c_v0 = c0 + c1 T */
    double wall_u[2][3];    /* LBM_BC_WALL: wall velocities at x = -1 ([0]) and x = nx ([1]) */
    double wall_T[2];       /* LBM_BC_WALL: wall temperatures */
    double sc_cmu, sc_ceta, sc_ck; /* shock-capturing numerical transport
                               (Section 4.4, eqs. shock_cap, shock_cap_k, r = 5):
                               mu, eta, k of each cell gain rho C_mu fS,
                               rho C_eta fS and rho c_s C_k fs, with fS, fs the
                               Gaussian-filtered (radius 4, sigma 1.2 cells)
                               |sum_a d^4/dx_a^4| of the strain-rate magnitude
                               S = |grad u + grad u^T| / 2 and of the entropy
                               gradient magnitude |grad s|.  All zero: off.
                               Non-zero coefficients take the multi-kernel
                               path (the extra passes need the fields of every
                               cell through HBM). */
} lbm_params;

typedef struct lbm_ctx lbm_ctx; /* opaque, library-owned */

/* Life cycle.  The problem statement's "initialise from (rho, u, T)" is split
 * in two calls so that the caller can hand over device arrays (torch tensors)
 * and reuse one context for several initial states: lbm_create validates the
 * parameters and allocates every device buffer the step needs; lbm_init fills
 * the populations; lbm_destroy releases the context.  No other call
 * allocates device memory except lbm_mlp_train and lbm_mlp_loss_grad (their
 * scratch, released before they return).
 *
 * Create a context: validates parameters and allocates the two population
 * buffers and the per-cell work arrays on the current device.
 * Errors: LBM_EINVAL (bad sizes, lattice, bc, storage/eos combination,
 * non-positive cv, mu; nz != 1 for lattice 2; check_every < 0), LBM_ENOMEM,
 * LBM_EDEVICE. */
int lbm_create(const lbm_params *params, lbm_ctx **out);

/* Release every device allocation of the context (NULL is accepted). */
void lbm_destroy(lbm_ctx *ctx);

/* Initialise f_i = f_i^eq(rho, u, theta), g_i = g_i^eq(rho, u, T, theta) with
 * theta = P(rho, T)/rho (flowchart "initialise"; eqs. LBMeq, LBMeqG).
 * dev_rho[N], dev_u[D*N], dev_T[N]: FP64 device arrays.  The inputs are
 * checked first (blocking): a non-finite value gives LBM_ENAN, a cell
 * outside the admissible set (see LBM_EUNSTABLE; P and theta from eq. Pvdw
 * at the cell's rho, T) gives LBM_EUNSTABLE, and the context is then left
 * uninitialised.  The initialisation itself is asynchronous.
 * Errors: LBM_EINVAL (NULL pointer), LBM_ENAN, LBM_EUNSTABLE, LBM_EDEVICE. */
int lbm_init(lbm_ctx *ctx, const double *dev_rho, const double *dev_u, const double *dev_T);

/* Advance n >= 0 full steps (collide + stream).  Asynchronous when
 * params.check_every is 0: non-finite or inadmissible states then surface
 * through lbm_conservation().  With check_every > 0 the state is checked after
 * every check_every-th step (a blocking fields pass and reduction); the first
 * failing check ends the call with LBM_ENAN or LBM_EUNSTABLE, the steps
 * before it having been taken.
 * Errors: LBM_ESTATE (not initialised), LBM_EINVAL (n < 0), LBM_ENAN,
 * LBM_EUNSTABLE, LBM_EDEVICE. */
int lbm_step(lbm_ctx *ctx, int n);

/* Macroscopic fields of the current state with the half-force corrections
 * (eqs. def_h, def_u, def_E, lbm_temp, Pvdw).  Any pointer may be NULL.
 * dev_rho[N], dev_u[D*N], dev_T[N], dev_P[N] FP64.  Asynchronous. */
int lbm_moments(lbm_ctx *ctx, double *dev_rho, double *dev_u, double *dev_T, double *dev_P);

/* Raw populations (decoded to FP64) of the current state, post-streaming at
 * time t; layout populations[i * N + idx].  Asynchronous. */
int lbm_get_populations(lbm_ctx *ctx, double *dev_f, double *dev_g);

/* Overwrite the state with the given FP64 populations (rounded to the
 * storage form).  Asynchronous.  Resume from lbm_get_populations output
 * reproduces the continuation bitwise for FP64/FP32 storage. */
int lbm_set_populations(lbm_ctx *ctx, const double *dev_f, const double *dev_g);

/* FP64 global sums of the current state, deterministic order (wavefront
 * reductions, fixed-order second pass).  host_out[D + 4] receives, in order:
 *   [0] sum rho, [1..D] sum (sum_i c_i f_i + F/2) = sum rho u,
 *   [D+1] sum_i g_i summed over cells, [D+2] number of non-finite cells,
 *   [D+3] number of finite cells outside the admissible set (LBM_EUNSTABLE).
 * Blocking (synchronises the stream).  Returns LBM_ENAN when [D+2] > 0,
 * else LBM_EUNSTABLE when [D+3] > 0 (the sums are written either way). */
int lbm_conservation(lbm_ctx *ctx, double *host_out);

/* Block until all work queued on the context's stream has finished. */
int lbm_synchronize(lbm_ctx *ctx);

/* Timed variant of lbm_step for measurement: runs n steps on the context's
 * stream with HIP events around every kernel launch and writes the average
 * duration in milliseconds of each kernel kind of the step to host_ms[k],
 * k < LBM_NUM_KERNELS (names from lbm_kernel_name; unused slots get "" and
 * 0).  Blocking.  Errors: as lbm_step; LBM_EINVAL when nslots <
 * LBM_NUM_KERNELS. */
#define LBM_NUM_KERNELS 4
int lbm_step_timed(lbm_ctx *ctx, int n, double *host_ms, int nslots);
const char *lbm_kernel_name(const lbm_ctx *ctx, int kernel);

/* 1 when lbm_step runs the single-pass fused kernel (one read and one write
 * of every population per step; periodic z or D = 2, and one plane of
 * populations, one moment layer and the inbound slots each below 2^31 bytes)
 * followed by the small pass completing its moment side channel (kernel kinds
 * "k_fused", "k_fused_fixup"; with the surrogate EOS the network runs in a
 * pass ahead of them, kind "k_eos_surrogate", writing the network's T of
 * every cell and whether it passed the residual check), 0 when
 * it runs the four-kernel path (moments, Laplacian, fields, collide). */
int lbm_is_fused(const lbm_ctx *ctx);

/* Algorithmic HBM bytes moved per cell update by lbm_step (2 Q populations
 * read + 2 Q written, in the storage width) -- the traffic an ideal fused
 * kernel needs, used for roofline accounting. */
double lbm_bytes_per_cell(const lbm_ctx *ctx);

const char *lbm_strerror(int status);

/* Text of the most recent failed HIP call seen by the library on the calling
 * thread ("" if none): the detail behind LBM_EDEVICE and LBM_ENOMEM. */
const char *lbm_last_error(void);

/* ---- learned equation-of-state surrogate ------------------------------- */
/* Network 2 -> 64 -> 64 -> 3 with ReLU hidden layers.  Parameter vector
 * (4547 FP32 values, LBM_MLP_NPARAMS):
 *   W1[64][2], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]
 * Normalisation vector (10 FP32 values, LBM_MLP_NNORM):
 *   lo_rho, hi_rho, lo_e, hi_e, mean_T, std_T, mean_P, std_P, mean_c2, std_c2
 * Inputs are scaled to [-1, 1]: xhat = 2 (x - lo)/(hi - lo) - 1; outputs are
 * yhat * std + mean.  The 64x64 layer runs on BF16 MFMA with FP32 accumulate
 * (LBM_MLP_BF16) or in FP32 on the vector ALU (LBM_MLP_F32); LBM_MLP_BF16_L1
 * (forward only) also runs the first layer on BF16 MFMA with the inputs and
 * its weights rounded to BF16 -- the form the step's surrogate pass uses. */
#define LBM_MLP_NPARAMS 4547
#define LBM_MLP_NNORM 10
#define LBM_MLP_BF16 0
#define LBM_MLP_F32 1
#define LBM_MLP_BF16_L1 2

/* Train a surrogate on the GPU with the library's own forward, backward and
 * Adam kernels.  Samples (rho, T) are drawn uniformly from the box
 * host_box = {rho_lo, rho_hi, T_lo, T_hi} by a counter-based generator
 * seeded with `seed`; targets (T, P, c_s^2) and inputs (rho, e) come from
 * the context-free van der Waals closed forms with the constants of params
 * (eqs. Pvdw, de_vdW, vdW_speed_of_sound).  MSE loss on z-scored outputs,
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8), learning rate lr with cosine
 * decay over `epochs` passes of n_samples / batch minibatches.
 * host_params[4547] (in: initial weights, out: trained), host_norm[10]
 * (out), host_loss (out, nullable: final epoch's mean loss).  Blocking.
 * Errors: LBM_EINVAL (n_samples < batch, batch not a multiple of 64). */
int lbm_mlp_train(const lbm_params *params, const double *host_box, int n_samples,
                  uint64_t seed, int epochs, int batch, float lr, int precision,
                  float *host_params, float *host_norm, double *host_loss);

/* Install a trained surrogate in a context created with eos = LBM_EOS_MLP.
 * host_params[4547], host_norm[10].  Blocking copy to device memory. */
int lbm_mlp_set(lbm_ctx *ctx, const float *host_params, const float *host_norm);

/* Fraction of cell evaluations since the last call that failed the residual
 * check and took the Newton fallback (blocking; resets the counters). */
int lbm_mlp_stats(lbm_ctx *ctx, double *host_fallback_fraction);

/* Statistics of the equation-of-state stage of the steps since the last call
 * (blocking; resets the counters): the fraction of surrogate evaluations
 * that failed the residual check (0 without the surrogate) and the mean
 * number of Peng-Robinson Newton iterations per cell update (0 for van der
 * Waals).  Either pointer may be NULL. */
int lbm_eos_stats(lbm_ctx *ctx, double *host_fallback_fraction, double *host_mean_newton_iterations);

/* Stand-alone surrogate forward pass: dev_x[2*B] raw (rho, e) pairs,
 * dev_y[3*B] de-normalised (T, P, c_s^2); dev_params[4547], dev_norm[10];
 * precision LBM_MLP_BF16, LBM_MLP_F32 or LBM_MLP_BF16_L1.
 * B >= 0 any size.  Asynchronous on `stream`. */
int lbm_mlp_forward(const float *dev_params, const float *dev_norm, const float *dev_x,
                    float *dev_y, int B, int precision, void *stream);

/* One Adam update of a parameter vector (the optimiser step of
 * lbm_mlp_train): m = b1 m + (1 - b1) grad, v = b2 v + (1 - b2) grad^2,
 * params -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + 1e-8) with
 * b1 = 0.9, b2 = 0.999 and t >= 1 the number of the update.  dev_params,
 * dev_m, dev_v (updated in place) and dev_grad: 4547 FP32 values each.
 * Asynchronous on `stream`.  Errors: LBM_EINVAL (NULL pointer, t < 1,
 * lr not positive). */
int lbm_mlp_adam(float *dev_params, const float *dev_grad, float *dev_m, float *dev_v, int t, float lr,
                 void *stream);

/* Mean-squared loss and its gradient on a batch: dev_xn[2*B] normalised
 * inputs, dev_tn[3*B] normalised targets (row-major per sample),
 * dev_grad[4547] (out), dev_loss[1] (out).  B a positive multiple of 64.
 * Asynchronous on `stream`. */
int lbm_mlp_loss_grad(const float *dev_params, const float *dev_xn, const float *dev_tn,
                      int B, float *dev_grad, float *dev_loss, int precision, void *stream);

/* lbm_mlp_loss_grad without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving or training loops,
 * harnesses that forbid hipMalloc.  Same arguments, kernels and results as
 * lbm_mlp_loss_grad (bit for bit), with B a positive multiple of 64 of at
 * most LBM_MLP_NOALLOC_MAX_BATCH.  The per-block partial sums live in a
 * library-owned static device array (2.3 MB on every GPU the library is
 * called on, kept until the process ends); each call overwrites the part it
 * uses before reading it.  Calls that overlap on one GPU (different streams
 * or threads) share that array and race: serialise them.  Asynchronous on
 * `stream` (no synchronisation).  The first call on a device looks up the
 * array's address there.  Errors: LBM_EINVAL (B out of range, precision,
 * NULL pointer), LBM_EDEVICE. */
#define LBM_MLP_NOALLOC_MAX_BATCH 8192
int lbm_mlp_loss_grad_noalloc(const float *dev_params, const float *dev_xn, const float *dev_tn, int B,
                              float *dev_grad, float *dev_loss, int precision, void *stream);

/* ---- HBM ceiling probe -------------------------------------------------- */
/* The practical bandwidth ceiling the step's kernels are measured against:
 * kind 0 reads `bytes` of dev_src, 1 writes `bytes` of dev_dst, 2 copies
 * dev_src to dev_dst; 16-byte accesses per lane with the non-temporal hint,
 * blocks_per_cu (1..64) workgroups of 256 threads per compute unit striding
 * over the buffer.  host_ms receives the average duration of `iters`
 * launches after one warm-up launch (HIP events; blocking).  Buffers are
 * caller-owned, `bytes` a multiple of 16 (dev_dst needs 16 bytes for kind 0).
 * Errors: LBM_EINVAL, LBM_EDEVICE. */
int lbm_hbm_probe(int kind, const void *dev_src, void *dev_dst, int64_t bytes, int blocks_per_cu, int iters,
                  void *stream, double *host_ms);

/* ---- precision codec ---------------------------------------------------- */
/* dev_out[n] = 16-bit code of dev_x[n] - dev_ref[n] (FP32 subtraction,
 * round-to-nearest-even; kind LBM_STORE_BF16 or LBM_STORE_F16); the decode
 * is dev_ref + code.  Asynchronous on `stream`. */
int lbm_codec_encode(int kind, const float *dev_x, const float *dev_ref, uint16_t *dev_out,
                     int64_t n, void *stream);
int lbm_codec_decode(int kind, const uint16_t *dev_code, const float *dev_ref, float *dev_out,
                     int64_t n, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
