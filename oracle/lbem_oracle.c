/*
 * lbem_oracle.c -- plain CPU reference for the two lattice-Boltzmann models of
 * Maxwell's equations compared in arXiv 2309.08068: the Mendoza-Munoz model
 * (MM, Section II) and the modified Hauser-Verhey model (HV, Section III).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark load this library.  The product (the HIP library)
 * shares no code with it and never calls it.
 *
 * What it computes, in the order of the pseudo-code of Appendix B:
 *   t = 0 : f := f_eq(E0, B0, J = 0)                      (initialisation)
 *   each step n (state f_n -> f_{n+1}):
 *     collision: moments -> constitutive relations and current -> equilibria
 *                -> BGK with tau = 1/2, f' = 2 f_eq - f (+ T for HV)
 *     imposition: hard-source cells get f' := f_eq(E_imp(n), B_imp(n), J = 0)
 *     advection:  f_{n+1}(x + v_q, q) = f'(x, q), periodic on every axis
 * Two arrays (read f_n, write f_{n+1}); no fusion beyond what the scheme says.
 *
 * Arithmetic is in `real`: double by default.  The library is also built once
 * with -DORACLE_REAL=float, only to measure how far single precision drifts
 * from double on the same scheme (the floor any FP32 implementation shares).
 *
 * Readings of points the paper leaves open (each is listed in the design notes
 * of the repository with its reason):
 *   - MM planes p = 0, 1, 2 as in eq. (VelocitySetMiller).
 *   - MM with both an ohmic and a prescribed current J_src:
 *       E = (D'/eps_r - mu0 J_src / (4 eps_r)) / (1 + mu0 sigma / (4 eps_r)),
 *       J = sigma E + J_src,
 *     which reduces to eqs. (MacroscopicEMiller) and (MacorscopicCurrentMiller)
 *     when either term vanishes.
 *   - MM rest population f_0^(1) is collided like f_0^(0) (eq. CollisionMiller
 *     writes only the latter; eq. equilibriumsMiller gives both equilibria).
 *   - MM H = B / (mu0 mu_r) (the constitutive relation of Section I-B with
 *     mu = mu_r mu0); used only for the reported H and the energy.
 *   - HV has no rest population (36 scalars, sums over i = 1..6).
 *   - HV lattice constants eps0 = mu0 = 3, so that the vacuum speed is 1/3.
 *   - HV current J = sigma E + J_src from the pre-collision D (no correction).
 *   - The fields of a state f_n are the pre-collision moments at the start of
 *     step n; MM reports the corrected E (eq. MacroscopicEMiller) using J_src(n).
 *   - Initial state: equilibrium with J = 0 and rho_c = 0.
 *   - Time dependent sources use the time level n of the state being collided.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORACLE_REAL
#define ORACLE_REAL double
#endif
typedef ORACLE_REAL real;

#define MODEL_MM 0
#define MODEL_HV 1
#define MM_Q 50
#define HV_Q 36
#define PI_D 3.14159265358979323846

/* lattice constants: MM eps0 = 1, mu0 = 2 (Section II-A); HV eps0 = mu0 = 3 */
static const real MM_EPS0 = 1, MM_MU0 = 2;
static const real HV_EPS0 = 3, HV_MU0 = 3;

/* ------------------------------------------------------------------------ */
/* MM vector sets, eqs. (VelocitySetMiller) and (ElectromagneticVectorsMiller) */
/* index [p][i-1] for plane p = 0..2 and direction i = 1..4, [j] for j = 0, 1  */
static int  mm_vi[3][4][3];
static real mm_v[3][4][3];
static real mm_e[3][4][2][3];
static real mm_b[3][4][2][3];
/* HV velocity set (Section III) */
static const int hv_vi[6][3] = {{1, 0, 0}, {0, 1, 0}, {-1, 0, 0},
                                {0, -1, 0}, {0, 0, -1}, {0, 0, 1}};
static int tables_ready = 0;

static void cross(const real a[3], const real b[3], real out[3]) {
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

static void build_tables(void) {
    if (tables_ready) return;
    for (int p = 0; p < 3; ++p)
        for (int i = 1; i <= 4; ++i) {
            double ang = (2.0 * i - 1.0) * PI_D / 4.0;
            double c = sqrt(2.0) * cos(ang), s = sqrt(2.0) * sin(ang);
            double v[3];
            if (p == 0) { v[0] = c; v[1] = s; v[2] = 0; }
            else if (p == 1) { v[0] = c; v[1] = 0; v[2] = s; }
            else { v[0] = 0; v[1] = c; v[2] = s; }
            /* the components are exactly -1, 0 or +1; remove the cos/sin rounding */
            for (int a = 0; a < 3; ++a) {
                mm_vi[p][i - 1][a] = (int)lround(v[a]);
                mm_v[p][i - 1][a] = (real)mm_vi[p][i - 1][a];
            }
        }
    for (int p = 0; p < 3; ++p)
        for (int i = 1; i <= 4; ++i) {
            int k0 = ((i + 2) % 4) + 1; /* e_{i0} = v_{[(i+2) mod 4]+1} / 2 */
            int k1 = (i % 4) + 1;       /* e_{i1} = v_{[i mod 4]+1} / 2     */
            for (int a = 0; a < 3; ++a) {
                mm_e[p][i - 1][0][a] = (real)0.5 * mm_v[p][k0 - 1][a];
                mm_e[p][i - 1][1][a] = (real)0.5 * mm_v[p][k1 - 1][a];
            }
            for (int j = 0; j < 2; ++j) cross(mm_v[p][i - 1], mm_e[p][i - 1][j], mm_b[p][i - 1][j]);
        }
    tables_ready = 1;
}

/* population index of f^{p(r)}_{ij}; 48 is f_0^(0), 49 is f_0^(1) */
static inline int mm_q(int r, int p, int i /*1..4*/, int j) { return r * 24 + p * 8 + (i - 1) * 2 + j; }
/* population index of component a of e_i (r = 0) or h_i (r = 1), i = 1..6 */
static inline int hv_q(int r, int i, int a) { return r * 18 + (i - 1) * 3 + a; }

/* ------------------------------------------------------------------------ */
/* MM single-cell pieces                                                      */

/* eq. (MacroscopicFieldsMiller) */
static void mm_moments(const real *f, real D[3], real B[3], real *rho) {
    D[0] = D[1] = D[2] = B[0] = B[1] = B[2] = 0;
    real r0 = f[48];
    for (int p = 0; p < 3; ++p)
        for (int i = 1; i <= 4; ++i)
            for (int j = 0; j < 2; ++j) {
                real f0 = f[mm_q(0, p, i, j)], f1 = f[mm_q(1, p, i, j)];
                for (int a = 0; a < 3; ++a) {
                    D[a] += f0 * mm_e[p][i - 1][j][a];
                    B[a] += f1 * mm_b[p][i - 1][j][a];
                }
                r0 += f0;
            }
    *rho = r0;
}

/* eqs. (MacroscopicEMiller), (MacorscopicCurrentMiller), joint reading above */
static void mm_macro(const real D[3], real eps_r, real sigma, const real Jsrc[3], real E[3], real J[3]) {
    real s = MM_MU0 * sigma / (4 * eps_r);
    for (int a = 0; a < 3; ++a) {
        E[a] = (D[a] / eps_r - MM_MU0 * Jsrc[a] / (4 * eps_r)) / (1 + s);
        J[a] = sigma * E[a] + Jsrc[a];
    }
}

static real dot3(const real a[3], const real b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* eq. (equilibriumsMiller) */
static void mm_equilibrium(const real E[3], const real B[3], const real J[3], real rho, real eps_r, real mu_r,
                           real *feq) {
    for (int p = 0; p < 3; ++p)
        for (int i = 1; i <= 4; ++i)
            for (int j = 0; j < 2; ++j) {
                real vJ = dot3(mm_v[p][i - 1], J) / 16;
                real Ee = dot3(E, mm_e[p][i - 1][j]);
                real Bb = dot3(B, mm_b[p][i - 1][j]);
                feq[mm_q(0, p, i, j)] = vJ + eps_r / 4 * Ee + Bb / (8 * mu_r);
                feq[mm_q(1, p, i, j)] = vJ + Ee / 4 + Bb / 8;
            }
    feq[48] = rho;
    feq[49] = rho;
}

/* ------------------------------------------------------------------------ */
/* HV single-cell pieces                                                      */

/* eq. (MacroscopicFieldsHV) */
static void hv_moments(const real *f, real D[3], real B[3]) {
    D[0] = D[1] = D[2] = B[0] = B[1] = B[2] = 0;
    for (int i = 1; i <= 6; ++i)
        for (int a = 0; a < 3; ++a) {
            D[a] += f[hv_q(0, i, a)];
            B[a] += f[hv_q(1, i, a)];
        }
}

/* eq. (equilibriumHV); D, B the moments, eps = eps0 eps_r, mu = mu0 mu_r */
static void hv_equilibrium(const real D[3], const real B[3], real eps, real mu, real *feq) {
    real Eo[3] = {D[0] / eps, D[1] / eps, D[2] / eps};
    real Ho[3] = {B[0] / mu, B[1] / mu, B[2] / mu};
    for (int i = 1; i <= 6; ++i) {
        real v[3] = {(real)hv_vi[i - 1][0], (real)hv_vi[i - 1][1], (real)hv_vi[i - 1][2]};
        real vxH[3], vxE[3];
        cross(v, Ho, vxH);
        cross(v, Eo, vxE);
        for (int a = 0; a < 3; ++a) {
            feq[hv_q(0, i, a)] = (D[a] - 3 * vxH[a]) / 6;
            feq[hv_q(1, i, a)] = (B[a] + 3 * vxE[a]) / 6;
        }
    }
}

/* eq. (SourceTermHV): T_i = -(J . v_i) v_i / 2, stored as [6][3] */
static void hv_source(const real J[3], real T[6][3]) {
    for (int i = 1; i <= 6; ++i) {
        real v[3] = {(real)hv_vi[i - 1][0], (real)hv_vi[i - 1][1], (real)hv_vi[i - 1][2]};
        real Jv = dot3(J, v);
        for (int a = 0; a < 3; ++a) T[i - 1][a] = -Jv * v[a] / 2;
    }
}

/* ------------------------------------------------------------------------ */
/* Exported single-cell operators (used by the identity and spectral tests)  */

int oracle_real_bytes(void) { return (int)sizeof(real); }
int oracle_threads(void) { return omp_get_max_threads(); }
int oracle_nq(int model) { return model == MODEL_MM ? MM_Q : (model == MODEL_HV ? HV_Q : -1); }

/* velocity of population q (integer components), for either model */
int oracle_velocity(int model, int q, int v[3]) {
    build_tables();
    if (model == MODEL_MM) {
        if (q < 0 || q >= MM_Q) return -1;
        if (q >= 48) { v[0] = v[1] = v[2] = 0; return 0; }
        int rem = q % 24, p = rem / 8, i = (rem % 8) / 2 + 1;
        for (int a = 0; a < 3; ++a) v[a] = mm_vi[p][i - 1][a];
        return 0;
    }
    if (model == MODEL_HV) {
        if (q < 0 || q >= HV_Q) return -1;
        int i = (q % 18) / 3 + 1;
        for (int a = 0; a < 3; ++a) v[a] = hv_vi[i - 1][a];
        return 0;
    }
    return -1;
}

/* MM vector tables as doubles: v[3][4][3], e[3][4][2][3], b[3][4][2][3] */
void oracle_mm_tables(double *v, double *e, double *b) {
    build_tables();
    for (int p = 0; p < 3; ++p)
        for (int i = 0; i < 4; ++i)
            for (int a = 0; a < 3; ++a) {
                v[(p * 4 + i) * 3 + a] = (double)mm_v[p][i][a];
                for (int j = 0; j < 2; ++j) {
                    e[((p * 4 + i) * 2 + j) * 3 + a] = (double)mm_e[p][i][j][a];
                    b[((p * 4 + i) * 2 + j) * 3 + a] = (double)mm_b[p][i][j][a];
                }
            }
}

/* equilibrium populations for given E, B, J (and rho_c for MM) */
int oracle_equilibrium(int model, const double *E, const double *B, const double *J, double rho, double eps_r,
                       double mu_r, double *feq_out) {
    build_tables();
    real e[3] = {(real)E[0], (real)E[1], (real)E[2]}, b[3] = {(real)B[0], (real)B[1], (real)B[2]};
    real j[3] = {(real)J[0], (real)J[1], (real)J[2]};
    real feq[MM_Q];
    if (model == MODEL_MM) {
        mm_equilibrium(e, b, j, (real)rho, (real)eps_r, (real)mu_r, feq);
        for (int q = 0; q < MM_Q; ++q) feq_out[q] = (double)feq[q];
        return 0;
    }
    if (model == MODEL_HV) {
        /* HV equilibria are written in D and B; J enters only through T */
        real eps = HV_EPS0 * (real)eps_r, mu = HV_MU0 * (real)mu_r;
        real D[3] = {eps * e[0], eps * e[1], eps * e[2]};
        hv_equilibrium(D, b, eps, mu, feq);
        for (int q = 0; q < HV_Q; ++q) feq_out[q] = (double)feq[q];
        return 0;
    }
    return -1;
}

/* HV source term T_i for a given J, out [6][3] */
void oracle_hv_source(const double *J, double *T_out) {
    real j[3] = {(real)J[0], (real)J[1], (real)J[2]}, T[6][3];
    hv_source(j, T);
    for (int i = 0; i < 6; ++i)
        for (int a = 0; a < 3; ++a) T_out[i * 3 + a] = (double)T[i][a];
}

/* Collision of one cell (no imposition): fout = C(f) for the given media and
 * prescribed current; also returns E, B (reported fields) and J. */
static void collide_cell(int model, const real *f, real eps_r, real mu_r, real sigma, const real Jsrc[3],
                         real *fout, real E[3], real B[3], real J[3], real Dout[3], real Hout[3]) {
    if (model == MODEL_MM) {
        real D[3], rho, feq[MM_Q];
        mm_moments(f, D, B, &rho);
        mm_macro(D, eps_r, sigma, Jsrc, E, J);
        mm_equilibrium(E, B, J, rho, eps_r, mu_r, feq);
        for (int q = 0; q < MM_Q; ++q) fout[q] = 2 * feq[q] - f[q];
        for (int a = 0; a < 3; ++a) {
            Dout[a] = MM_EPS0 * eps_r * E[a];
            Hout[a] = B[a] / (MM_MU0 * mu_r);
        }
    } else {
        real D[3], feq[HV_Q], T[6][3];
        real eps = HV_EPS0 * eps_r, mu = HV_MU0 * mu_r;
        hv_moments(f, D, B);
        for (int a = 0; a < 3; ++a) {
            E[a] = D[a] / eps;
            J[a] = sigma * E[a] + Jsrc[a];
            Dout[a] = D[a];
            Hout[a] = B[a] / mu;
        }
        hv_equilibrium(D, B, eps, mu, feq);
        hv_source(J, T);
        for (int i = 1; i <= 6; ++i)
            for (int a = 0; a < 3; ++a) {
                int qe = hv_q(0, i, a), qh = hv_q(1, i, a);
                fout[qe] = 2 * feq[qe] - f[qe] + T[i - 1][a];
                fout[qh] = 2 * feq[qh] - f[qh];
            }
    }
}

int oracle_collide(int model, const double *f, double eps_r, double mu_r, double sigma, const double *Jsrc,
                   double *fout, double *E, double *B, double *J) {
    build_tables();
    int Q = oracle_nq(model);
    if (Q < 0) return -1;
    real fi[MM_Q], fo[MM_Q], js[3] = {(real)Jsrc[0], (real)Jsrc[1], (real)Jsrc[2]};
    real e[3], b[3], j[3], d[3], h[3];
    for (int q = 0; q < Q; ++q) fi[q] = (real)f[q];
    collide_cell(model, fi, (real)eps_r, (real)mu_r, (real)sigma, js, fo, e, b, j, d, h);
    for (int q = 0; q < Q; ++q) fout[q] = (double)fo[q];
    for (int a = 0; a < 3; ++a) {
        if (E) E[a] = (double)e[a];
        if (B) B[a] = (double)b[a];
        if (J) J[a] = (double)j[a];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The lattice problem                                                        */

typedef struct {
    int32_t model;
    int32_t nx, ny, nz;
    const double *eps_r, *mu_r, *sigma; /* [N] each; NULL means 1, 1, 0 */
    /* soft point currents: J_src(cell, n) = J0 sin(2 pi n / period + phase) */
    int32_t n_src;
    const int64_t *src_cell;   /* [n_src] linear cell index x + nx (y + ny z) */
    const double *src_J0;      /* [n_src][3] */
    const double *src_period;  /* [n_src] */
    const double *src_phase;   /* [n_src] */
    /* hard plane source at z = plane_z (< 0: none):
     * E_imp(n) = E0 sin(2 pi n / period), B_imp(n) = B0 sin(2 pi n / period) */
    int32_t plane_z;
    double plane_E0[3], plane_B0[3], plane_period;
} oracle_problem;

typedef struct {
    /* probes: E and B at given cells for every step, out [nsteps][n_probe][6] */
    int32_t n_probe;
    const int64_t *probe_cell;
    double *probe_series;
    /* detector: sum over the plane z = det_z of |E|^2 for every step, out [nsteps] */
    int32_t det_z; /* < 0: none */
    double *det_series;
    /* energy U = 1/2 sum (E.D + B.H) every energy_every steps, out [nsteps / every] */
    int32_t energy_every; /* <= 0: none */
    double *energy_series;
} oracle_observe;

static inline real medium(const double *a, int64_t c, real dflt) { return a ? (real)a[c] : dflt; }

/* index of the point current in cell c, or -1; built once per call */
static int32_t *source_map(const oracle_problem *P, int64_t N) {
    if (P->n_src <= 0) return NULL;
    int32_t *m = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    for (int64_t c = 0; c < N; ++c) m[c] = -1;
    for (int s = 0; s < P->n_src; ++s) {
        int64_t c = P->src_cell[s];
        if (c < 0 || c >= N || m[c] >= 0) { free(m); return (int32_t *)-1; } /* out of range or repeated */
        m[c] = s;
    }
    return m;
}

static void source_current(const oracle_problem *P, const int32_t *map, int64_t c, int64_t n, real J[3]) {
    J[0] = J[1] = J[2] = 0;
    int s = map ? map[c] : -1;
    if (s < 0) return;
    double w = sin(2.0 * PI_D * (double)n / P->src_period[s] + P->src_phase[s]);
    for (int a = 0; a < 3; ++a) J[a] = (real)(P->src_J0[3 * s + a] * w);
}

/* equilibrium used for initialisation and for hard sources (J = 0, rho_c = 0) */
static void field_equilibrium(int model, const real E[3], const real B[3], real eps_r, real mu_r, real *feq) {
    if (model == MODEL_MM) {
        real J[3] = {0, 0, 0};
        mm_equilibrium(E, B, J, 0, eps_r, mu_r, feq);
    } else {
        real eps = HV_EPS0 * eps_r, mu = HV_MU0 * mu_r;
        real D[3] = {eps * E[0], eps * E[1], eps * E[2]};
        hv_equilibrium(D, B, eps, mu, feq);
    }
}

/* periodic wrap of a coordinate that is at most one cell outside [0, n) */
static inline int64_t wrap(int64_t a, int64_t n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

/* f := f_eq(E0, B0, J = 0) in every cell; E0, B0 are [3][N] */
int oracle_init(const oracle_problem *P, const double *E0, const double *B0, real *f) {
    build_tables();
    int Q = oracle_nq(P->model);
    if (Q < 0 || P->nx < 1 || P->ny < 1 || P->nz < 1) return -1;
    int64_t N = (int64_t)P->nx * P->ny * P->nz;
    for (int64_t c = 0; c < N; ++c) {
        real E[3], B[3], feq[MM_Q];
        for (int a = 0; a < 3; ++a) {
            E[a] = (real)E0[a * N + c];
            B[a] = (real)B0[a * N + c];
        }
        field_equilibrium(P->model, E, B, medium(P->eps_r, c, 1), medium(P->mu_r, c, 1), feq);
        for (int q = 0; q < Q; ++q) f[q * N + c] = feq[q];
    }
    return 0;
}

/* reported fields of state f at time level n; any output may be NULL; [3][N] */
int oracle_fields(const oracle_problem *P, const real *f, int64_t n, double *E, double *B, double *D, double *H) {
    build_tables();
    int Q = oracle_nq(P->model);
    if (Q < 0) return -1;
    int64_t N = (int64_t)P->nx * P->ny * P->nz;
    int32_t *map = source_map(P, N);
    if (map == (int32_t *)-1) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        real fc[MM_Q], fo[MM_Q], e[3], b[3], j[3], d[3], h[3], js[3];
        for (int q = 0; q < Q; ++q) fc[q] = f[q * N + c];
        source_current(P, map, c, n, js);
        collide_cell(P->model, fc, medium(P->eps_r, c, 1), medium(P->mu_r, c, 1), medium(P->sigma, c, 0), js, fo, e,
                     b, j, d, h);
        for (int a = 0; a < 3; ++a) {
            if (E) E[a * N + c] = (double)e[a];
            if (B) B[a * N + c] = (double)b[a];
            if (D) D[a * N + c] = (double)d[a];
            if (H) H[a * N + c] = (double)h[a];
        }
    }
    free(map);
    return 0;
}

/* Advance nsteps steps starting at time level n0: f (in) -> f (out).
 * scratch must hold Q * N reals (the second lattice).  Observation of the
 * state f_n is taken before its collision, for n = n0 .. n0 + nsteps - 1. */
int oracle_run(const oracle_problem *P, real *f, real *scratch, int64_t n0, int64_t nsteps, const oracle_observe *O) {
    build_tables();
    const int model = P->model;
    const int Q = oracle_nq(model);
    if (Q < 0 || P->nx < 1 || P->ny < 1 || P->nz < 1 || nsteps < 0) return -1;
    const int64_t nx = P->nx, ny = P->ny, nz = P->nz, N = nx * ny * nz;
    int vel[MM_Q][3];
    for (int q = 0; q < Q; ++q) oracle_velocity(model, q, vel[q]);
    int32_t *map = source_map(P, N);
    if (map == (int32_t *)-1) return -1;
    double *cell_energy = NULL, *cell_det = NULL;
    int64_t plane_n = nx * ny;
    if (O && O->energy_every > 0) cell_energy = (double *)malloc(sizeof(double) * N);
    if (O && O->det_z >= 0) cell_det = (double *)malloc(sizeof(double) * plane_n);

    real *src = f, *dst = scratch;
    for (int64_t s = 0; s < nsteps; ++s) {
        const int64_t n = n0 + s;
        const int want_energy = cell_energy && (s % O->energy_every == 0);
        /* hard-source fields at this time level */
        real Eimp[3] = {0, 0, 0}, Bimp[3] = {0, 0, 0};
        if (P->plane_z >= 0) {
            double w = sin(2.0 * PI_D * (double)n / P->plane_period);
            for (int a = 0; a < 3; ++a) {
                Eimp[a] = (real)(P->plane_E0[a] * w);
                Bimp[a] = (real)(P->plane_B0[a] * w);
            }
        }
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    const int64_t c = x + nx * (y + ny * z);
                    real fc[MM_Q], fo[MM_Q], E[3], B[3], J[3], D[3], H[3], js[3];
                    const real er = medium(P->eps_r, c, 1), mr = medium(P->mu_r, c, 1), sg = medium(P->sigma, c, 0);
                    for (int q = 0; q < Q; ++q) fc[q] = src[q * N + c];
                    source_current(P, map, c, n, js);
                    /* collision */
                    collide_cell(model, fc, er, mr, sg, js, fo, E, B, J, D, H);
                    /* observation of the pre-collision state f_n */
                    if (want_energy) cell_energy[c] = 0.5 * (double)(dot3(E, D) + dot3(B, H));
                    if (cell_det && z == O->det_z) cell_det[x + nx * y] = (double)dot3(E, E);
                    if (O && O->n_probe > 0)
                        for (int k = 0; k < O->n_probe; ++k)
                            if (O->probe_cell[k] == c) {
                                double *o = O->probe_series + (s * O->n_probe + k) * 6;
                                for (int a = 0; a < 3; ++a) {
                                    o[a] = (double)E[a];
                                    o[3 + a] = (double)B[a];
                                }
                            }
                    /* imposition of the hard source */
                    if (P->plane_z >= 0 && z == P->plane_z) field_equilibrium(model, Eimp, Bimp, er, mr, fo);
                    /* advection */
                    for (int q = 0; q < Q; ++q) {
                        int64_t xd = wrap(x + vel[q][0], nx), yd = wrap(y + vel[q][1], ny), zd = wrap(z + vel[q][2], nz);
                        dst[q * N + xd + nx * (yd + ny * zd)] = fo[q];
                    }
                }
        if (want_energy) {
            double u = 0;
            for (int64_t c = 0; c < N; ++c) u += cell_energy[c];
            O->energy_series[s / O->energy_every] = u;
        }
        if (cell_det) {
            double u = 0;
            for (int64_t c = 0; c < plane_n; ++c) u += cell_det[c];
            O->det_series[s] = u;
        }
        real *t = src;
        src = dst;
        dst = t;
    }
    if (src != f) memcpy(f, src, sizeof(real) * (size_t)Q * (size_t)N);
    free(cell_energy);
    free(cell_det);
    free(map);
    return 0;
}
