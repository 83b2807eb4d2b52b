/*
 * Oracle of the non-ideal compressible double-distribution lattice Boltzmann
 * step (Hosseini, Feinberg & Karlin, arXiv 2510.14712, Section 3.2).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, scalar FP64 C
 * implementation written from the paper's equations.  It shares no code,
 * header, table or constant with the GPU library; only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.
 *
 * Conventions (all lattice units: dx = dt = 1, lattice speed c = 1,
 * lattice sound speed squared 1/3, quasi-equilibrium relaxation time = dt):
 *   - D = 2 (D2Q9) or D = 3 (D3Q27); velocity index
 *       i = (c_x + 1) + 3 (c_y + 1) [+ 9 (c_z + 1)],  c_a in {-1, 0, 1}.
 *   - cell index idx = x + nx (y + ny z), x fastest; nz = 1 when D = 2.
 *   - populations are structure-of-arrays: f[i * N + idx], N = nx ny nz.
 *   - vector fields likewise: u[a * N + idx].
 *   - boundary per axis: 0 periodic, 1 zero-gradient (indices clamped to the
 *     domain for both streaming and finite differences).
 *   - the stored state is the post-streaming population set at time t.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int D;              /* 2 or 3 */
    int nx, ny, nz;     /* nz must be 1 for D = 2 */
    int bc[3];          /* per axis: 0 periodic, 1 zero-gradient, 2 wall
                           (x axis only; see wall_u, wall_T) */
    double a, b, R, cv; /* van der Waals constants and isochoric heat */
    double mu, eta, k;  /* shear, bulk viscosity, thermal conductivity */
    double kappa;       /* capillarity coefficient */
    double upwind_eps;  /* |u_a| <= upwind_eps takes the central average in the
                           upwind-biased derivative of Lambda (sgn(u) = 0) */
    double sc_cmu, sc_ceta, sc_ck; /* coefficients C_mu, C_eta, C_k of the
                           shock-capturing numerical transport (Section 4.4);
                           all zero: off */
    int eos;            /* 0: van der Waals (a, b, R, cv); 1: Peng-Robinson
                           with a, b, R and the fields below (cv unused) */
    double pr_m, pr_Tc; /* Peng-Robinson alpha(T) = (1 + m (1 - sqrt(T/Tc)))^2 */
    double pr_c0, pr_c1; /* ideal-gas heat capacity c_v0(T) = c0 + c1 T */
    double wall_u[2][3]; /* wall velocities at x = -1 ([0]) and x = nx ([1]) */
    double wall_T[2];    /* wall temperatures there */
} oracle_params;

/* Per-cell fields produced while evaluating one step (all length N or D*N). */
typedef struct {
    double *rho, *u, *E, *T, *P, *theta, *h, *cs2, *F, *Lambda, *lap;
    double *Phi; /* Phi_aa = -(1/rho) d_a Lambda_a (upwind), D*N; filled by
                    oracle_collide only */
    double *mu_num, *eta_num, *k_num; /* numerical transport of each cell
                    (zero when shock capturing is off), N each */
} oracle_fields;

/* f = f^eq(rho, u, theta), g = g^eq(rho, u, T, theta), theta = P(rho,T)/rho. */
int oracle_init(const oracle_params *p, const double *rho, const double *u,
                const double *T, double *f, double *g);

/* Macroscopic fields of the current state (any pointer may be NULL). */
int oracle_fields_eval(const oracle_params *p, const double *f, const double *g,
                       oracle_fields *out);

/* Collision only: fpost/gpost receive the post-collision populations at the
 * same cell (no streaming).  out (nullable) receives the fields used. */
int oracle_collide(const oracle_params *p, const double *f, const double *g,
                   double *fpost, double *gpost, oracle_fields *out);

/* Pull streaming of post-collision populations into the state arrays
 * (periodic and zero-gradient axes; a wall axis needs the fields of the step
 * and is streamed by oracle_run: returns -1). */
int oracle_stream(const oracle_params *p, const double *fpost,
                  const double *gpost, double *f, double *g);

/* n full steps (collide + stream) in place on f, g. */
int oracle_run(const oracle_params *p, double *f, double *g, int nsteps);

/* Equation of state of the parameters at (rho, T): out[0] P, out[1] e,
 * out[2] c_v = (de/dT)_rho, out[3] c_s^2, out[4] (dP/dT)_rho. */
void oracle_eos(const oracle_params *p, double rho, double T, double *out);
/* Caloric inversion: T with e(rho, T) = e (explicit for van der Waals,
 * Newton iterations to convergence for Peng-Robinson).  Returns the number
 * of Newton iterations taken (0 for the explicit inversion), or -1 when the
 * iteration failed to converge. */
int oracle_temperature(const oracle_params *p, double rho, double e, double *T);

/* Equilibria of a single state (for moment tests). feq, geq: Q values.
 * e is the specific internal energy e(rho, T). */
void oracle_feq(int D, double rho, const double *u, double theta, double *feq);
void oracle_geq(int D, double rho, const double *u, double e, double theta,
                double *geq);
/* Operator moments M_k = prod_a O_a^{k_a} E, k_a in {0,1,2}, E = e + |u|^2/2,
 * O_a = theta d/du_a + u_a; output ordered k = k_x + 3 k_y (+ 9 k_z). */
void oracle_operator_moments(int D, const double *u, double e, double theta,
                             double *M);

int oracle_num_threads(void);
/* threads of the OpenMP loops over cells (n > 0) */
void oracle_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
