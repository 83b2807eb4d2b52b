/*
 * Oracle of the non-ideal compressible double-distribution lattice Boltzmann
 * step (arXiv 2510.14712, Section 3.2 "Lattice Boltzmann realization" and the
 * flowchart figure at its end).
 *
 * TEST INFRASTRUCTURE ONLY: plain scalar FP64, no blocking or fusion beyond
 * what the paper's equations state.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library; it shares nothing
 * with the GPU path.
 *
 * Each pass below names the equation it evaluates.  Where the paper is
 * ambiguous the reading taken is stated next to the code (the list of
 * readings is kept with the design notes of the repository).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LATTICE_SOUND_SPEED_SQ (1.0 / 3.0) /* varsigma^2, eq. (cs) */

/* ---------------------------------------------------------------------- */
/* Velocity set: c_{i a} in {-1,0,1}, i = (c_x+1) + 3(c_y+1) [+ 9(c_z+1)]  */
/* (eq. D3Q27c; D2Q9 is the same product restricted to two axes).          */
/* ---------------------------------------------------------------------- */
static int num_vel(int D) { return D == 2 ? 9 : 27; }

static void vel(int D, int i, int c[3]) {
    c[0] = i % 3 - 1;
    c[1] = (i / 3) % 3 - 1;
    c[2] = D == 3 ? (i / 9) - 1 : 0;
}

/* Psi_{i a}(xi, zeta) = 1 - c^2 + [(3c^2 - 2) zeta + c xi] / 2   (eq. phi) */
static double Psi(int c, double xi, double zeta) {
    double c2 = (double)(c * c);
    return 1.0 - c2 + 0.5 * ((3.0 * c2 - 2.0) * zeta + (double)c * xi);
}

/* ---------------------------------------------------------------------- */
/* f^eq (eq. LBMeq): rho * prod_a Psi(c_ia; u_a, theta + u_a^2)            */
/* ---------------------------------------------------------------------- */
void oracle_feq(int D, double rho, const double *u, double theta, double *feq) {
    int Q = num_vel(D);
    for (int i = 0; i < Q; i++) {
        int c[3];
        vel(D, i, c);
        double prod = 1.0;
        for (int a = 0; a < D; a++) prod *= Psi(c[a], u[a], theta + u[a] * u[a]);
        feq[i] = rho * prod;
    }
}

/* ---------------------------------------------------------------------- */
/* g^eq (eqs. Egen, Oa, LBMeqG): the product of Psi with xi -> O_a and     */
/* zeta -> O_a^2 acting on the generating function E = e + |u|^2/2.        */
/* The operators are applied literally to E held as a polynomial in the    */
/* velocity components; the result is evaluated at the given velocity.     */
/* ---------------------------------------------------------------------- */
#define PD 5 /* per-variable degree bound: E has degree 2, O_a^2 adds 2 */
typedef struct { double c[PD][PD][PD]; } poly3;

/* out = O_a in = theta * d(in)/du_a + u_a * in */
static void poly_apply_O(const poly3 *in, poly3 *out, int a, double theta) {
    memset(out, 0, sizeof(*out));
    for (int i = 0; i < PD; i++)
        for (int j = 0; j < PD; j++)
            for (int k = 0; k < PD; k++) {
                double v = in->c[i][j][k];
                if (v == 0.0) continue;
                int e[3] = {i, j, k};
                int n = e[a];
                if (n > 0) { /* derivative term */
                    int d[3] = {i, j, k};
                    d[a] = n - 1;
                    out->c[d[0]][d[1]][d[2]] += theta * (double)n * v;
                }
                /* multiplication by u_a; the degree bound is never exceeded
                 * for at most two applications per axis on E */
                int m[3] = {i, j, k};
                m[a] = n + 1;
                if (m[a] < PD) out->c[m[0]][m[1]][m[2]] += v;
                else abort();
            }
}

static double poly_eval(const poly3 *p, const double *u) {
    double pw[3][PD];
    for (int a = 0; a < 3; a++) {
        pw[a][0] = 1.0;
        for (int n = 1; n < PD; n++) pw[a][n] = pw[a][n - 1] * u[a];
    }
    double s = 0.0;
    for (int i = 0; i < PD; i++)
        for (int j = 0; j < PD; j++)
            for (int k = 0; k < PD; k++)
                if (p->c[i][j][k] != 0.0) s += p->c[i][j][k] * pw[0][i] * pw[1][j] * pw[2][k];
    return s;
}

void oracle_operator_moments(int D, const double *u, double e, double theta, double *M) {
    double uu[3] = {u[0], u[1], D == 3 ? u[2] : 0.0};
    poly3 E;
    memset(&E, 0, sizeof(E));
    E.c[0][0][0] = e;         /* e(rho, T) */
    E.c[2][0][0] += 0.5;      /* u_x^2 / 2 */
    E.c[0][2][0] += 0.5;      /* u_y^2 / 2 */
    if (D == 3) E.c[0][0][2] += 0.5;
    int nz = D == 3 ? 3 : 1;
    poly3 Pz[3], Pyz[3][3], t;
    Pz[0] = E;
    if (D == 3) {
        poly_apply_O(&Pz[0], &Pz[1], 2, theta);
        poly_apply_O(&Pz[1], &Pz[2], 2, theta);
    }
    for (int kz = 0; kz < nz; kz++) {
        Pyz[0][kz] = Pz[kz];
        poly_apply_O(&Pyz[0][kz], &Pyz[1][kz], 1, theta);
        poly_apply_O(&Pyz[1][kz], &Pyz[2][kz], 1, theta);
        for (int ky = 0; ky < 3; ky++) {
            poly3 cur = Pyz[ky][kz];
            for (int kx = 0; kx < 3; kx++) {
                if (kx > 0) {
                    poly_apply_O(&cur, &t, 0, theta);
                    cur = t;
                }
                M[kx + 3 * ky + 9 * kz] = poly_eval(&cur, uu);
            }
        }
    }
}

/* Weight of O^k inside Psi(c; O, O^2): constant term (1 - c^2) for k = 0,
 * c/2 for k = 1 and (3c^2 - 2)/2 for k = 2 (eq. phi). */
static double psi_weight(int c, int k) {
    double c2 = (double)(c * c);
    if (k == 0) return 1.0 - c2;
    if (k == 1) return 0.5 * (double)c;
    return 0.5 * (3.0 * c2 - 2.0);
}

void oracle_geq(int D, double rho, const double *u, double e, double theta, double *geq) {
    int Q = num_vel(D);
    double M[27];
    oracle_operator_moments(D, u, e, theta, M);
    int nk = D == 3 ? 27 : 9;
    for (int i = 0; i < Q; i++) {
        int c[3];
        vel(D, i, c);
        double s = 0.0;
        for (int kk = 0; kk < nk; kk++) {
            int k[3] = {kk % 3, (kk / 3) % 3, kk / 9};
            double w = 1.0;
            for (int a = 0; a < D; a++) w *= psi_weight(c[a], k[a]);
            s += w * M[kk];
        }
        geq[i] = rho * s;
    }
}

/* ---------------------------------------------------------------------- */
/* Equation of state.  van der Waals (eq. Pvdw with the caloric relation of */
/* eq. de_vdW, e = c_v T - a rho; its inversion is explicit, eq. lbm_temp), */
/* or Peng-Robinson, the paper's example of an equation of state whose     */
/* caloric relation must be inverted iteratively at every node (Section     */
/* 3.2, after eq. lbm_temp), written from Peng & Robinson's published form: */
/*   P = rho R T / (1 - b rho) - a alpha(T) rho^2 / (1 + 2 b rho - b^2 rho^2) */
/*   alpha(T) = (1 + m (1 - s))^2,  s = sqrt(T / Tc),                       */
/* with a temperature-dependent ideal-gas heat capacity c_v0 = c0 + c1 T.   */
/* The energy follows from the thermodynamic identity                      */
/*   (de/drho)_T = (P - T (dP/dT)_rho) / rho^2                              */
/* integrated from the dilute limit:                                        */
/*   e = c0 T + c1 T^2 / 2 - a (alpha - T alpha') L(rho),                   */
/*   alpha - T alpha' = (1 + m)(1 + m (1 - s)),                             */
/*   L(rho) = ln[(1 + (1 + sqrt2) b rho) / (1 + (1 - sqrt2) b rho)] / (2 sqrt2 b), */
/* quartic in s, hence Newton's method.  The adiabatic sound speed is the   */
/* general identity c_s^2 = (dP/drho)_T + T (dP/dT)_rho^2 / (rho^2 c_v)     */
/* (eq. speed_of_sound).                                                    */
/* ---------------------------------------------------------------------- */
static double pr_L(double b, double rho) {
    const double r2 = sqrt(2.0);
    return log((1.0 + (1.0 + r2) * b * rho) / (1.0 + (1.0 - r2) * b * rho)) / (2.0 * r2 * b);
}

void oracle_eos(const oracle_params *p, double rho, double T, double *out) {
    if (p->eos == 0) {
        double omb = 1.0 - p->b * rho;
        out[0] = rho * p->R * T / omb - p->a * rho * rho;                        /* eq. Pvdw */
        out[1] = p->cv * T - p->a * rho;                                          /* eq. de_vdW */
        out[2] = p->cv;
        out[3] = p->R * T * (1.0 + p->R / p->cv) / (omb * omb) - 2.0 * p->a * rho; /* eq. vdW_speed_of_sound */
        out[4] = rho * p->R / omb;
        return;
    }
    const double a = p->a, b = p->b, R = p->R, m = p->pr_m;
    const double s = sqrt(T / p->pr_Tc);
    const double k = 1.0 + m * (1.0 - s);
    const double alpha = k * k;
    const double dalpha = -m * k / sqrt(T * p->pr_Tc);          /* d alpha / dT */
    const double d2alpha = 0.5 * m * (1.0 + m) / (T * sqrt(T * p->pr_Tc)); /* d^2 alpha / dT^2 */
    const double den = 1.0 + 2.0 * b * rho - b * b * rho * rho;
    const double omb = 1.0 - b * rho;
    const double L = pr_L(b, rho);
    out[0] = rho * R * T / omb - a * alpha * rho * rho / den;
    out[1] = p->pr_c0 * T + 0.5 * p->pr_c1 * T * T - a * (1.0 + m) * k * L;
    out[2] = p->pr_c0 + p->pr_c1 * T + a * T * d2alpha * L;     /* c_v0 + a T alpha'' L */
    out[4] = rho * R / omb - a * dalpha * rho * rho / den;
    const double dPdrho = R * T / (omb * omb) - a * alpha * (2.0 * rho * den - rho * rho * (2.0 * b - 2.0 * b * b * rho)) / (den * den);
    out[3] = dPdrho + T * out[4] * out[4] / (rho * rho * out[2]);
}

int oracle_temperature(const oracle_params *p, double rho, double e, double *T) {
    if (p->eos == 0) {
        *T = (e + p->a * rho) / p->cv;                               /* eq. lbm_temp */
        return 0;
    }
    /* Newton's method on e(rho, T) - e = 0 from the dilute (ideal-gas)
     * estimate c0 T = e, kept positive by halving a step that would not be */
    double t = e / p->pr_c0;
    if (!(t > 1e-3 * p->pr_Tc)) t = p->pr_Tc;
    double q[5];
    for (int it = 1; it <= 100; it++) {
        oracle_eos(p, rho, t, q);
        double dt = (q[1] - e) / q[2];
        double tn = t - dt;
        while (!(tn > 0.0)) {
            dt *= 0.5;
            tn = t - dt;
        }
        t = tn;
        if (fabs(dt) <= 1e-15 * t) {
            *T = t;
            return it;
        }
    }
    *T = t;
    return -1;
}

/* ---------------------------------------------------------------------- */
/* Grid helpers                                                            */
/* ---------------------------------------------------------------------- */
static int check_params(const oracle_params *p) {
    if (!p) return -1;
    if (p->eos != 0 && p->eos != 1) return -1;
    if (p->eos == 1 && !(p->pr_Tc > 0 && p->pr_c0 > 0)) return -1;
    if (p->D != 2 && p->D != 3) return -1;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
    if (p->D == 2 && p->nz != 1) return -1;
    for (int a = 0; a < 3; a++)
        if (p->bc[a] != 0 && p->bc[a] != 1 && !(p->bc[a] == 2 && a == 0)) return -1;
    if (p->bc[0] == 2 && (p->bc[1] != 0 || p->bc[2] != 0)) return -1; /* walls: periodic y, z */
    return 0;
}

static int coord(int x, int n, int bc) {
    if (x >= 0 && x < n) return x;
    if (bc == 0) return ((x % n) + n) % n; /* periodic */
    return x < 0 ? 0 : n - 1;               /* zero-gradient (and wall): clamp */
}

/* index of the cell at (x, y, z) + (dx, dy, dz) under the boundary rules */
static long nbr(const oracle_params *p, long idx, int dx, int dy, int dz) {
    int x = (int)(idx % p->nx);
    int y = (int)((idx / p->nx) % p->ny);
    int z = (int)(idx / ((long)p->nx * p->ny));
    int X = coord(x + dx, p->nx, p->bc[0]);
    int Y = coord(y + dy, p->ny, p->bc[1]);
    int Z = coord(z + dz, p->nz, p->bc[2]);
    return X + (long)p->nx * (Y + (long)p->ny * Z);
}

static long nbr_axis(const oracle_params *p, long idx, int a, int s) {
    int d[3] = {0, 0, 0};
    d[a] = s;
    return nbr(p, idx, d[0], d[1], d[2]);
}

/* ---------------------------------------------------------------------- */
/* Walls (bc 2 on the x axis), for the thermal Couette flow of Section 4.1, */
/* whose wall treatment the paper does not state.  Reading: diffuse         */
/* reflection.  Each ghost cell beyond a wall (x = -1, x = nx) absorbs the  */
/* populations that leave the domain into it and re-emits equilibria of the */
/* wall state -- velocity u_w, temperature T_w, and the thermodynamic state */
/* of the boundary cell next to it (theta_w = P(rho_b, T_w)/rho_b, e_w =    */
/* e(rho_b, T_w)) -- scaled so that the ghost emits the mass it absorbed    */
/* (no mass crosses the wall).  The central differences of u, T, h and      */
/* Lambda at the boundary cell take the ghost's values (with rho_b); rho    */
/* and its Laplacian, and the shock-capturing stencils, stay zero-gradient. */
/* ---------------------------------------------------------------------- */
typedef struct {
    double u[3], T, theta, e, h;
} ghost_state;

static ghost_state wall_ghost(const oracle_params *p, int side, double rho_g) {
    ghost_state gs;
    double q[5];
    for (int a = 0; a < 3; a++) gs.u[a] = p->wall_u[side][a];
    gs.T = p->wall_T[side];
    oracle_eos(p, rho_g, gs.T, q);
    gs.theta = q[0] / rho_g;
    gs.e = q[1];
    gs.h = gs.e + gs.theta;
    return gs;
}

/* side of the wall the neighbour x + s e_a lies beyond (0 low, 1 high), or -1 */
static int beyond_wall(const oracle_params *p, long idx, int a, int s) {
    if (a != 0 || p->bc[0] != 2) return -1;
    int x = (int)(idx % p->nx) + s;
    return x < 0 ? 0 : (x >= p->nx ? 1 : -1);
}

/* ---------------------------------------------------------------------- */
/* Macroscopic fields of a state: flowchart boxes "compute rho and F" and  */
/* "compute u, E, T, P" (eqs. def_h, FK, def_u, def_E, lbm_temp, Pvdw).    */
/* ---------------------------------------------------------------------- */
typedef struct {
    double *rho, *J, *G, *lap, *F, *u, *E, *T, *P, *theta, *e, *h, *cs2, *Lam;
    double *Phi; /* diagonal Galilean correction of each cell, set by the collision */
    double *mu_num, *eta_num, *k_num; /* shock-capturing numerical transport */
    double *sc_a, *sc_b;              /* scratch of the shock-capturing passes */
    double *cv, *dPdT;                /* c_v and (dP/dT)_rho of each cell */
} work_fields;

static void shock_capturing(const oracle_params *p, work_fields *w);

static void work_alloc(work_fields *w, long N, int D) {
    w->rho = calloc(N, sizeof(double));
    w->J = calloc((size_t)D * N, sizeof(double));
    w->G = calloc(N, sizeof(double));
    w->lap = calloc(N, sizeof(double));
    w->F = calloc((size_t)D * N, sizeof(double));
    w->u = calloc((size_t)D * N, sizeof(double));
    w->E = calloc(N, sizeof(double));
    w->T = calloc(N, sizeof(double));
    w->P = calloc(N, sizeof(double));
    w->theta = calloc(N, sizeof(double));
    w->e = calloc(N, sizeof(double));
    w->h = calloc(N, sizeof(double));
    w->cs2 = calloc(N, sizeof(double));
    w->Lam = calloc((size_t)D * N, sizeof(double));
    w->Phi = calloc((size_t)D * N, sizeof(double));
    w->mu_num = calloc(N, sizeof(double));
    w->eta_num = calloc(N, sizeof(double));
    w->k_num = calloc(N, sizeof(double));
    w->sc_a = calloc(N, sizeof(double));
    w->sc_b = calloc(N, sizeof(double));
    w->cv = calloc(N, sizeof(double));
    w->dPdT = calloc(N, sizeof(double));
}

static void work_free(work_fields *w) {
    free(w->rho); free(w->J); free(w->G); free(w->lap); free(w->F); free(w->u);
    free(w->E); free(w->T); free(w->P); free(w->theta); free(w->e); free(w->h);
    free(w->cs2); free(w->Lam); free(w->Phi);
    free(w->mu_num); free(w->eta_num); free(w->k_num); free(w->sc_a); free(w->sc_b);
    free(w->cv); free(w->dPdT);
}

static void compute_fields(const oracle_params *p, const double *f, const double *g,
                           work_fields *w) {
    const int D = p->D, Q = num_vel(D);
    const long N = (long)p->nx * p->ny * p->nz;

    /* rho = sum f_i (eq. def_h); sum c_i f_i and sum g_i enter eqs. def_u, def_E */
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double rho = 0.0, J[3] = {0.0, 0.0, 0.0}, G = 0.0;
        for (int i = 0; i < Q; i++) {
            int c[3];
            vel(D, i, c);
            rho += f[i * N + x];
            for (int a = 0; a < D; a++) J[a] += (double)c[a] * f[i * N + x];
            G += g[i * N + x];
        }
        w->rho[x] = rho;
        for (int a = 0; a < D; a++) w->J[a * N + x] = J[a];
        w->G[x] = G;
    }

    /* Laplacian of rho by the central second-order difference per axis */
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double s = 0.0;
        for (int a = 0; a < D; a++)
            s += w->rho[nbr_axis(p, x, a, +1)] + w->rho[nbr_axis(p, x, a, -1)] - 2.0 * w->rho[x];
        w->lap[x] = s;
    }

    /* Korteweg force F = kappa rho grad(lap rho)  (eq. FK), central gradient */
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        for (int a = 0; a < D; a++) {
            double d = 0.5 * (w->lap[nbr_axis(p, x, a, +1)] - w->lap[nbr_axis(p, x, a, -1)]);
            w->F[a * N + x] = p->kappa * w->rho[x] * d;
        }
    }

    /* u, E, T, P and the derived per-cell quantities */
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double rho = w->rho[x];
        double u[3] = {0.0, 0.0, 0.0}, uF = 0.0, u2 = 0.0;
        for (int a = 0; a < D; a++) {
            u[a] = (w->J[a * N + x] + 0.5 * w->F[a * N + x]) / rho; /* eq. def_u */
            uF += u[a] * w->F[a * N + x];
            u2 += u[a] * u[a];
        }
        double E = (w->G[x] + 0.5 * uF) / rho;                  /* eq. def_E */
        double e = E - 0.5 * u2;                                /* eq. rhoE */
        double T, q[5];
        oracle_temperature(p, rho, e, &T);                      /* eq. lbm_temp, or Newton */
        oracle_eos(p, rho, T, q);
        double P = q[0];                                        /* eq. Pvdw (or Peng-Robinson) */
        double theta = P / rho;                                 /* eq. theta */
        double h = e + P / rho;                                 /* eq. enthalpy */
        double cs2 = q[3];
        w->cv[x] = q[2];
        w->dPdT[x] = q[4];
        for (int a = 0; a < D; a++) {
            w->u[a * N + x] = u[a];
            /* Lambda_a = rho u_a^3 + 3 rho u_a (theta - varsigma^2) */
            w->Lam[a * N + x] = rho * u[a] * u[a] * u[a] + 3.0 * rho * u[a] * (theta - LATTICE_SOUND_SPEED_SQ);
        }
        w->E[x] = E; w->T[x] = T; w->P[x] = P; w->theta[x] = theta;
        w->e[x] = e; w->h[x] = h; w->cs2[x] = cs2;
    }

    /* numerical transport of the shock-capturing scheme (zero when off) */
    shock_capturing(p, w);
}

/* ---------------------------------------------------------------------- */
/* Shock-capturing numerical transport (Section 4.4, eqs. shock_cap and   */
/* shock_cap_k): with r = 5 and dx = 1                                     */
/*   {mu, eta}^num = rho C_{mu,eta} filt(|grad^4 S|),                      */
/*   k^num         = rho c_s C_k   filt(|grad^4 |grad s||),                */
/*   S = (1/2) sqrt((grad u + grad u^T) : (grad u + grad u^T)),            */
/*   grad s = (c_v / T) grad T - R / (rho (1 - b rho)) grad rho            */
/* (entropy gradient of van der Waals, from eq. ds_vdW).  Readings where   */
/* the paper is silent: grad^4 phi = sum_a d^4 phi / dx_a^4 by the central */
/* fourth difference along each axis; first derivatives central; the       */
/* filter is a separable truncated Gaussian, weights exp(-j^2/(2 sigma^2)) */
/* for |j| <= 4 with sigma = 1.2 cells, normalised to sum one, applied     */
/* along x, then y, then z; c_s = sqrt(max(c_s^2, 0)).                     */
/* ---------------------------------------------------------------------- */
#define SC_FILTER_RADIUS 4
#define SC_FILTER_SIGMA 1.2

static int sc_enabled(const oracle_params *p) {
    return p->sc_cmu != 0.0 || p->sc_ceta != 0.0 || p->sc_ck != 0.0;
}

/* |sum_a (phi(x+2e_a) - 4 phi(x+e_a) + 6 phi(x) - 4 phi(x-e_a) + phi(x-2e_a))| */
static void abs_fourth_difference(const oracle_params *p, const double *phi, double *out) {
    const long N = (long)p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double s = 0.0;
        for (int a = 0; a < p->D; a++) {
            long p1 = nbr_axis(p, x, a, 1), p2 = nbr_axis(p, x, a, 2);
            long m1 = nbr_axis(p, x, a, -1), m2 = nbr_axis(p, x, a, -2);
            s += phi[p2] - 4.0 * phi[p1] + 6.0 * phi[x] - 4.0 * phi[m1] + phi[m2];
        }
        out[x] = fabs(s);
    }
}

/* in place: phi <- Gaussian filter of phi along each axis in turn (tmp: scratch) */
static void gaussian_filter(const oracle_params *p, double *phi, double *tmp) {
    const long N = (long)p->nx * p->ny * p->nz;
    double wts[2 * SC_FILTER_RADIUS + 1], wsum = 0.0;
    for (int j = -SC_FILTER_RADIUS; j <= SC_FILTER_RADIUS; j++) {
        wts[j + SC_FILTER_RADIUS] = exp(-(double)(j * j) / (2.0 * SC_FILTER_SIGMA * SC_FILTER_SIGMA));
        wsum += wts[j + SC_FILTER_RADIUS];
    }
    for (int j = 0; j <= 2 * SC_FILTER_RADIUS; j++) wts[j] /= wsum;
    for (int a = 0; a < p->D; a++) {
#pragma omp parallel for schedule(static)
        for (long x = 0; x < N; x++) {
            double s = 0.0;
            for (int j = -SC_FILTER_RADIUS; j <= SC_FILTER_RADIUS; j++)
                s += wts[j + SC_FILTER_RADIUS] * phi[nbr_axis(p, x, a, j)];
            tmp[x] = s;
        }
        memcpy(phi, tmp, (size_t)N * sizeof(double));
    }
}

static void shock_capturing(const oracle_params *p, work_fields *w) {
    const int D = p->D;
    const long N = (long)p->nx * p->ny * p->nz;
    if (!sc_enabled(p)) {
        memset(w->mu_num, 0, (size_t)N * sizeof(double));
        memset(w->eta_num, 0, (size_t)N * sizeof(double));
        memset(w->k_num, 0, (size_t)N * sizeof(double));
        return;
    }
    /* strain-rate magnitude S into sc_a */
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double G[3][3] = {{0}}; /* G[a][b] = d u_a / d x_b */
        for (int b = 0; b < D; b++) {
            long xp = nbr_axis(p, x, b, 1), xm = nbr_axis(p, x, b, -1);
            for (int a = 0; a < D; a++) G[a][b] = 0.5 * (w->u[a * N + xp] - w->u[a * N + xm]);
        }
        double ss = 0.0;
        for (int a = 0; a < D; a++)
            for (int b = 0; b < D; b++) ss += (G[a][b] + G[b][a]) * (G[a][b] + G[b][a]);
        w->sc_a[x] = 0.5 * sqrt(ss);
    }
    abs_fourth_difference(p, w->sc_a, w->mu_num);
    gaussian_filter(p, w->mu_num, w->sc_b);
    /* entropy-gradient magnitude |grad s| into sc_a */
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double rho = w->rho[x], T = w->T[x], g2 = 0.0;
        for (int a = 0; a < D; a++) {
            long xp = nbr_axis(p, x, a, 1), xm = nbr_axis(p, x, a, -1);
            double dT = 0.5 * (w->T[xp] - w->T[xm]), dr = 0.5 * (w->rho[xp] - w->rho[xm]);
            /* ds = (c_v / T) dT - (dP/dT)_rho / rho^2 drho; van der Waals:
             * (dP/dT)_rho / rho^2 = R / (rho (1 - b rho)) */
            double ds = p->eos == 0 ? p->cv / T * dT - p->R / (rho * (1.0 - p->b * rho)) * dr
                                    : w->cv[x] / T * dT - w->dPdT[x] / (rho * rho) * dr;
            g2 += ds * ds;
        }
        w->sc_a[x] = sqrt(g2);
    }
    abs_fourth_difference(p, w->sc_a, w->k_num);
    gaussian_filter(p, w->k_num, w->sc_b);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double rho = w->rho[x], fS = w->mu_num[x];
        double cs = sqrt(w->cs2[x] > 0.0 ? w->cs2[x] : 0.0);
        w->mu_num[x] = rho * p->sc_cmu * fS;
        w->eta_num[x] = rho * p->sc_ceta * fS;
        w->k_num[x] = rho * cs * p->sc_ck * w->k_num[x];
    }
}

static void export_fields(const oracle_params *p, const work_fields *w, oracle_fields *out) {
    if (!out) return;
    const long N = (long)p->nx * p->ny * p->nz;
    const int D = p->D;
#define CP(dst, src, n) if (out->dst) memcpy(out->dst, w->src, (size_t)(n) * sizeof(double))
    CP(rho, rho, N); CP(u, u, D * N); CP(E, E, N); CP(T, T, N); CP(P, P, N);
    CP(theta, theta, N); CP(h, h, N); CP(cs2, cs2, N); CP(F, F, D * N);
    CP(Lambda, Lam, D * N); CP(lap, lap, N); CP(Phi, Phi, D * N);
    CP(mu_num, mu_num, N); CP(eta_num, eta_num, N); CP(k_num, k_num, N);
#undef CP
}

/* sgn with a dead zone: |v| <= eps counts as zero, which takes the central
 * average (reading of the tie sgn(0); the upwind switch is discontinuous at
 * u = 0, so velocities at round-off level must not pick a side) */
static double sgn(double v, double eps) { return v > eps ? 1.0 : (v < -eps ? -1.0 : 0.0); }

/* ---------------------------------------------------------------------- */
/* Collision (eqs. fLBGK, gLBGK with LBMeq, LBMstar, LBMeqG, LBMgstar)     */
/* ---------------------------------------------------------------------- */
static void collide_all(const oracle_params *p, const double *f, const double *g,
                        work_fields *w, double *fpost, double *gpost) {
    const int D = p->D, Q = num_vel(D);
    const long N = (long)p->nx * p->ny * p->nz;

#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double rho = w->rho[x], P = w->P[x], theta = w->theta[x], T = w->T[x];
        double u[3] = {0, 0, 0}, F[3] = {0, 0, 0};
        for (int a = 0; a < D; a++) { u[a] = w->u[a * N + x]; F[a] = w->F[a * N + x]; }

        /* central differences: div u, grad h, grad T */
        double divu = 0.0, gh[3] = {0, 0, 0}, gT[3] = {0, 0, 0}, Phi[3] = {0, 0, 0};
        for (int a = 0; a < D; a++) {
            long xp = nbr_axis(p, x, a, +1), xm = nbr_axis(p, x, a, -1);
            /* u_a, h, T, Lambda_a at x - e_a (index 0) and x + e_a (1): the
             * neighbours', or a wall ghost's */
            double nu[2] = {w->u[a * N + xm], w->u[a * N + xp]};
            double nh[2] = {w->h[xm], w->h[xp]}, nT[2] = {w->T[xm], w->T[xp]};
            double nL[2] = {w->Lam[a * N + xm], w->Lam[a * N + xp]};
            for (int k = 0; k < 2; k++) {
                int side = beyond_wall(p, x, a, k ? 1 : -1);
                if (side < 0) continue;
                ghost_state gs = wall_ghost(p, side, rho);
                nu[k] = gs.u[a];
                nh[k] = gs.h;
                nT[k] = gs.T;
                nL[k] = rho * gs.u[a] * gs.u[a] * gs.u[a] + 3.0 * rho * gs.u[a] * (gs.theta - LATTICE_SOUND_SPEED_SQ);
            }
            divu += 0.5 * (nu[1] - nu[0]);
            gh[a] = 0.5 * (nh[1] - nh[0]);
            gT[a] = 0.5 * (nT[1] - nT[0]);
            /* upwind-biased derivative of Lambda_a by the sign of u_a at x,
             * then Phi_aa = -(1/rho) d_a Lambda_a (eq. correction) */
            double s = sgn(u[a], p->upwind_eps);
            double dL = 0.5 * (1.0 + s) * (w->Lam[a * N + x] - nL[0])
                      + 0.5 * (1.0 - s) * (nL[1] - w->Lam[a * N + x]);
            Phi[a] = -dL / rho;
            w->Phi[a * N + x] = Phi[a];
        }

        /* transport coefficients with the numerical contributions (zero
         * without shock capturing), Section 4.4 */
        double mu = p->mu + w->mu_num[x], eta = p->eta + w->eta_num[x], kk = p->k + w->k_num[x];
        double tau = mu / P;                                            /* tau = mu / P */
        double beta = 1.0 / (2.0 * tau + 1.0);                         /* eq. beta_main, dt = 1 */
        double alpha = (double)(D + 2) / (double)D - rho * w->cs2[x] / P - eta / mu; /* eq. corr_bulk */

        double us[3] = {0, 0, 0}, FF = 0.0;
        for (int a = 0; a < D; a++) { us[a] = u[a] + F[a] / rho; FF += F[a] * F[a]; } /* eq. sh_vel_1 */
        double thetas = theta + alpha * theta * divu;                  /* eq. sh_temp_1 */
        double Ts = T - FF / (2.0 * rho * rho * w->cv[x]);             /* eq. sh_T_1 */
        double qc[3] = {0, 0, 0};
        for (int a = 0; a < D; a++) qc[a] = P * (gh[a] - (kk / mu) * gT[a]); /* eq. qc_1 */

        double q[5];
        oracle_eos(p, rho, T, q);
        double e_eq = q[1];                     /* caloric EOS e(rho, T) (eq. de_vdW) */
        /* e(rho, T*): van der Waals by its caloric relation at T*; for an
         * energy non-linear in T the value the shift stands for,
         * e - |F|^2 / (2 rho^2) (equal to e(rho, T*) to O(|F|^4), and exact
         * for van der Waals), so that the collision changes sum_i g_i by
         * exactly u . F */
        double e_st;
        if (p->eos == 0) {
            oracle_eos(p, rho, Ts, q);
            e_st = q[1];
        } else {
            e_st = e_eq - FF / (2.0 * rho * rho);
        }

        double feq[27], fst[27], geq[27], gst[27];
        oracle_feq(D, rho, u, theta, feq);
        for (int i = 0; i < Q; i++) {           /* eq. LBMstar */
            int c[3];
            vel(D, i, c);
            double prod = 1.0;
            for (int a = 0; a < D; a++) prod *= Psi(c[a], us[a], thetas + us[a] * us[a] + Phi[a]);
            fst[i] = rho * prod;
        }
        oracle_geq(D, rho, u, e_eq, theta, geq);
        oracle_geq(D, rho, us, e_st, thetas, gst);
        for (int i = 0; i < Q; i++) {           /* eq. LBMgstar: + c_i.q^c / 2 on |c_i|^2 = 1 */
            int c[3];
            vel(D, i, c);
            int c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
            if (c2 == 1) {
                double cq = 0.0;
                for (int a = 0; a < D; a++) cq += (double)c[a] * qc[a];
                gst[i] += 0.5 * cq;
            }
        }
        for (int i = 0; i < Q; i++) {
            double fi = f[i * N + x], gi = g[i * N + x];
            fpost[i * N + x] = fi + 2.0 * beta * (feq[i] - fi) + (1.0 - beta) * (fst[i] - feq[i]);
            gpost[i * N + x] = gi + 2.0 * beta * (geq[i] - gi) + (1.0 - beta) * (gst[i] - geq[i]);
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Public entry points                                                     */
/* ---------------------------------------------------------------------- */
int oracle_init(const oracle_params *p, const double *rho, const double *u,
                const double *T, double *f, double *g) {
    if (check_params(p)) return -1;
    const int D = p->D, Q = num_vel(D);
    const long N = (long)p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double r = rho[x], t = T[x], uu[3] = {0, 0, 0}, q[5];
        for (int a = 0; a < D; a++) uu[a] = u[a * N + x];
        oracle_eos(p, r, t, q);
        double P = q[0];
        double theta = P / r;
        double e = q[1];
        double feq[27], geq[27];
        oracle_feq(D, r, uu, theta, feq);
        oracle_geq(D, r, uu, e, theta, geq);
        for (int i = 0; i < Q; i++) { f[i * N + x] = feq[i]; g[i * N + x] = geq[i]; }
    }
    return 0;
}

int oracle_fields_eval(const oracle_params *p, const double *f, const double *g,
                       oracle_fields *out) {
    if (check_params(p)) return -1;
    const long N = (long)p->nx * p->ny * p->nz;
    work_fields w;
    work_alloc(&w, N, p->D);
    compute_fields(p, f, g, &w);
    export_fields(p, &w, out);
    work_free(&w);
    return 0;
}

int oracle_collide(const oracle_params *p, const double *f, const double *g,
                   double *fpost, double *gpost, oracle_fields *out) {
    if (check_params(p)) return -1;
    const long N = (long)p->nx * p->ny * p->nz;
    work_fields w;
    work_alloc(&w, N, p->D);
    compute_fields(p, f, g, &w);
    collide_all(p, f, g, &w, fpost, gpost);
    export_fields(p, &w, out);
    work_free(&w);
    return 0;
}

/* the populations a wall ghost emits replace what the clamped pull read:
 * f_i(x) for x - c_i beyond the wall comes from the ghost at x - c_i.  That
 * ghost absorbed the post-collision populations f'_j (pointing out through
 * the wall) of the boundary cells x_g - c_j (x_g: the ghost's position) and
 * emits m / s times the equilibria of the wall state at the boundary cell
 * next to it, where m is the absorbed mass and s the sum of the emitted
 * equilibria per unit density */
static void wall_inflow(const oracle_params *p, const work_fields *w, const double *fpost, double *f, double *g) {
    const int D = p->D, Q = num_vel(D);
    const long N = (long)p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        for (int i = 0; i < Q; i++) {
            int c[3];
            vel(D, i, c);
            int side = beyond_wall(p, x, 0, -c[0]);
            if (side < 0) continue;
            /* the ghost sits at x - c_i; the boundary cell next to it is the
             * same position with x clamped into the domain */
            long adj = nbr(p, x, -c[0], -c[1], -c[2]);
            double rho_b = w->rho[adj];
            ghost_state gs = wall_ghost(p, side, rho_b);
            /* absorbed mass: populations j with c_jx pointing through this
             * wall, from the boundary cells adj - (c_jy, c_jz) */
            double m = 0.0;
            for (int j = 0; j < Q; j++) {
                int cj[3];
                vel(D, j, cj);
                if (cj[0] != -c[0]) continue;
                long src = nbr(p, adj, 0, -cj[1], -cj[2]);
                m += fpost[j * N + src];
            }
            double feq[27], geq[27], sm = 0.0;
            oracle_feq(D, 1.0, gs.u, gs.theta, feq);
            for (int j = 0; j < Q; j++) {
                int cj[3];
                vel(D, j, cj);
                if (cj[0] == c[0]) sm += feq[j];
            }
            double rho_g = m / sm;
            oracle_feq(D, rho_g, gs.u, gs.theta, feq);
            oracle_geq(D, rho_g, gs.u, gs.e, gs.theta, geq);
            f[i * N + x] = feq[i];
            g[i * N + x] = geq[i];
        }
    }
}

static int stream_pull(const oracle_params *p, const double *fpost, const double *gpost, double *f, double *g);

int oracle_stream(const oracle_params *p, const double *fpost, const double *gpost,
                  double *f, double *g) {
    if (check_params(p) || p->bc[0] == 2) return -1;
    return stream_pull(p, fpost, gpost, f, g);
}

static int stream_pull(const oracle_params *p, const double *fpost, const double *gpost,
                       double *f, double *g) {
    const int D = p->D, Q = num_vel(D);
    const long N = (long)p->nx * p->ny * p->nz;
    /* f_i(x + c_i, t + 1) = f'_i(x, t), written as a pull from x - c_i */
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        for (int i = 0; i < Q; i++) {
            int c[3];
            vel(D, i, c);
            long src = nbr(p, x, -c[0], -c[1], -c[2]);
            f[i * N + x] = fpost[i * N + src];
            g[i * N + x] = gpost[i * N + src];
        }
    }
    return 0;
}

int oracle_run(const oracle_params *p, double *f, double *g, int nsteps) {
    if (check_params(p) || nsteps < 0) return -1;
    const int Q = num_vel(p->D);
    const long N = (long)p->nx * p->ny * p->nz;
    double *fp = malloc((size_t)Q * N * sizeof(double));
    double *gp = malloc((size_t)Q * N * sizeof(double));
    if (!fp || !gp) { free(fp); free(gp); return -2; }
    work_fields w;
    work_alloc(&w, N, p->D);
    for (int s = 0; s < nsteps; s++) {
        compute_fields(p, f, g, &w);
        collide_all(p, f, g, &w, fp, gp);
        stream_pull(p, fp, gp, f, g);
        if (p->bc[0] == 2) wall_inflow(p, &w, fp, f, g);
    }
    work_free(&w);
    free(fp);
    free(gp);
    return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
