/*
 * nh_oracle.c -- plain FP64 CPU oracle for the element-based Galerkin
 * nonhydrostatic model (Kang, Giraldo & Camp, arXiv 2504.08157).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * What it computes (all FP64, plain loops, no blocking or fusion):
 *   - LGL nodes, weights and the Lagrange derivative matrix (Sec. 2.2, basis
 *     functions and quadrature rule).
 *   - The hexahedral mesh: element->unique map "intma" (Algorithm 1), node
 *     coordinates, and the diagonal mass M_I, assembled by direct stiffness
 *     summation of the element masses (Sec. 2.2, mass matrix equation).
 *   - The element tendency  r = w_i w_j w_k J^e S(q)  at every local node:
 *     global-to-local gather, reference-space gradients (Algorithm 2),
 *     divergence of the momentum, metric terms, sources (Eq. governing),
 *     then the DSS gather (Algorithm 3, done serially in ascending element
 *     and node order, so results do not depend on the thread count) and the
 *     mass inverse (Eq. governing:matrix).
 *   - SSP-RK3 time stepping.
 *   - The standalone DSS (Algorithm 3) and local scatter.
 *   - The vertical linear operator L_v of a 1D-IMEX (HEVI) split, applied on
 *     the unique lattice (Sec. 2.3, IMEX splitting S = (S - L) + L).
 *
 * Readings of the paper (where it is silent) are documented next to the code
 * that applies them.  Parity of everything here is pinned by the CPU tests.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NF 5 /* prognostic fields: rho', u, v, w, theta' (Sec. 2.1) */
#define MAXN 8
#define MAXNP ((MAXN + 1) * (MAXN + 1) * (MAXN + 1))

/* ------------------------------------------------------------------ */
/* Legendre polynomial P_n(x) and its derivative, by the three-term     */
/* recurrence (textbook definition).                                    */
/* ------------------------------------------------------------------ */
static void legendre(int n, double x, double *p, double *dp)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *p = p1;
    /* P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1), valid off the endpoints */
    if (fabs(x) < 1.0)
        *dp = n * (x * p1 - p0) / (x * x - 1.0);
    else
        *dp = 0.5 * n * (n + 1.0) * (x > 0 ? 1.0 : ((n % 2) ? 1.0 : -1.0));
}

/*
 * LGL points (Sec. 2.2: tensor-product Lagrange basis on Legendre-Gauss-Lobatto
 * points).  xi_0 = -1, xi_N = 1; interior points are the roots of P_N'.
 * Weights w_j = 2 / (N (N+1) P_N(xi_j)^2).  D_ij = h_j'(xi_i) with the
 * classical closed form for LGL Lagrange polynomials.
 * D is row-major: D[i*(N+1)+j].
 */
int or_lgl(int N, double *xi, double *w, double *D)
{
    if (N < 1 || N > 16) return -1;
    int n1 = N + 1;
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        /* Newton on P_N'(x) = 0, start from the Chebyshev-Gauss-Lobatto point */
        double x = -cos(M_PI * j / N);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(N, x, &p, &dp);
            /* P_N'' from the Legendre ODE: (1-x^2) P'' = 2x P' - N(N+1) P */
            double ddp = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
            double dx = dp / ddp;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        xi[j] = x;
    }
    /* exact mirror symmetry of the node set */
    for (int j = 0; j < n1 / 2; ++j) {
        double a = 0.5 * (xi[N - j] - xi[j]);
        xi[j] = -a;
        xi[N - j] = a;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    double pn[17];
    for (int j = 0; j < n1; ++j) {
        double p, dp;
        legendre(N, xi[j], &p, &dp);
        pn[j] = p;
        w[j] = 2.0 / (N * (N + 1.0) * p * p);
    }
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) {
            double d;
            if (i != j)
                d = pn[i] / (pn[j] * (xi[i] - xi[j]));
            else if (i == 0)
                d = -0.25 * N * (N + 1.0);
            else if (i == N)
                d = 0.25 * N * (N + 1.0);
            else
                d = 0.0;
            D[i * n1 + j] = d;
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Oracle context                                                      */
/* ------------------------------------------------------------------ */
typedef struct {
    int nsnap;
    double *t;     /* [nsnap] */
    double *vals;  /* [nsnap][U] */
} forcing_t;

typedef struct {
    int N, n1, np;          /* order, N+1, (N+1)^3 */
    int nel[3], per[2];
    int n[3];               /* lattice sizes */
    int64_t E, L, U;
    double *xe, *ye, *ze;   /* element edges */
    double xi[17], w[17], D[17 * 17];
    int64_t *intma;         /* [L] */
    double *M;              /* [U] */
    double *lx, *ly, *lz;   /* lattice coordinates per direction */
    /* physics */
    double g, R, cp, cv, pa, fcor, zs, taumax;
    /* reference state per level */
    double *rho0, *theta0, *p0, *tau; /* [n_z] */
    forcing_t frc[NF];
    double *work;           /* [NF][L] element tendencies */
} or_ctx;

static double lattice_coord(const double *edges, int nel, int N, const double *xi,
                            int periodic, int idx)
{
    int e = idx / N, i = idx % N;
    if (!periodic && e == nel) { e = nel - 1; i = N; }
    if (i == 0) return edges[e];
    if (i == N) return edges[e + 1];
    double h = edges[e + 1] - edges[e];
    return edges[e] + 0.5 * h * (xi[i] + 1.0);
}

void or_destroy(void *p);

void *or_create(int N, const int *nel, const double *xe, const double *ye,
                const double *ze, const int *per)
{
    if (N < 1 || N > MAXN) return NULL;
    for (int d = 0; d < 3; ++d) if (nel[d] < 1) return NULL;
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    c->N = N;
    c->n1 = N + 1;
    c->np = c->n1 * c->n1 * c->n1;
    for (int d = 0; d < 3; ++d) c->nel[d] = nel[d];
    c->per[0] = per[0];
    c->per[1] = per[1];
    c->n[0] = nel[0] * N + (per[0] ? 0 : 1);
    c->n[1] = nel[1] * N + (per[1] ? 0 : 1);
    c->n[2] = nel[2] * N + 1;
    c->E = (int64_t)nel[0] * nel[1] * nel[2];
    c->L = c->E * c->np;
    c->U = (int64_t)c->n[0] * c->n[1] * c->n[2];
    c->xe = (double *)malloc(sizeof(double) * (nel[0] + 1));
    c->ye = (double *)malloc(sizeof(double) * (nel[1] + 1));
    c->ze = (double *)malloc(sizeof(double) * (nel[2] + 1));
    memcpy(c->xe, xe, sizeof(double) * (nel[0] + 1));
    memcpy(c->ye, ye, sizeof(double) * (nel[1] + 1));
    memcpy(c->ze, ze, sizeof(double) * (nel[2] + 1));
    or_lgl(N, c->xi, c->w, c->D);

    /* intma: local node (i,j,k) of element e -> unique lattice node (Algorithm 1) */
    c->intma = (int64_t *)malloc(sizeof(int64_t) * c->L);
    for (int ez = 0; ez < nel[2]; ++ez)
        for (int ey = 0; ey < nel[1]; ++ey)
            for (int ex = 0; ex < nel[0]; ++ex) {
                int64_t e = ex + (int64_t)nel[0] * (ey + (int64_t)nel[1] * ez);
                for (int k = 0; k < c->n1; ++k)
                    for (int j = 0; j < c->n1; ++j)
                        for (int i = 0; i < c->n1; ++i) {
                            int ix = ex * N + i, iy = ey * N + j, iz = ez * N + k;
                            if (per[0]) ix %= c->n[0];
                            if (per[1]) iy %= c->n[1];
                            c->intma[e * c->np + i + c->n1 * (j + c->n1 * k)] =
                                ix + (int64_t)c->n[0] * (iy + (int64_t)c->n[1] * iz);
                        }
            }

    c->lx = (double *)malloc(sizeof(double) * c->n[0]);
    c->ly = (double *)malloc(sizeof(double) * c->n[1]);
    c->lz = (double *)malloc(sizeof(double) * c->n[2]);
    for (int i = 0; i < c->n[0]; ++i) c->lx[i] = lattice_coord(xe, nel[0], N, c->xi, per[0], i);
    for (int i = 0; i < c->n[1]; ++i) c->ly[i] = lattice_coord(ye, nel[1], N, c->xi, per[1], i);
    for (int i = 0; i < c->n[2]; ++i) c->lz[i] = lattice_coord(ze, nel[2], N, c->xi, 0, i);

    /* diagonal mass: DSS of w_i w_j w_k J^e (Sec. 2.2, mass matrix; inexact
       LGL integration makes it diagonal).  Accumulated in ascending
       (e, k, j, i) order. */
    c->M = (double *)calloc(c->U, sizeof(double));
    for (int64_t e = 0; e < c->E; ++e) {
        int ex = (int)(e % nel[0]), ey = (int)((e / nel[0]) % nel[1]), ez = (int)(e / ((int64_t)nel[0] * nel[1]));
        double J = (xe[ex + 1] - xe[ex]) * (ye[ey + 1] - ye[ey]) * (ze[ez + 1] - ze[ez]) / 8.0;
        for (int k = 0; k < c->n1; ++k)
            for (int j = 0; j < c->n1; ++j)
                for (int i = 0; i < c->n1; ++i)
                    c->M[c->intma[e * c->np + i + c->n1 * (j + c->n1 * k)]] +=
                        c->w[i] * c->w[j] * c->w[k] * J;
    }

    /* default physics (overridden by or_set_physics) */
    c->g = 9.80616; c->cp = 1004.67; c->cv = 717.5; c->R = c->cp - c->cv; c->pa = 1.0e5;
    c->rho0 = (double *)calloc(c->n[2], sizeof(double));
    c->theta0 = (double *)calloc(c->n[2], sizeof(double));
    c->p0 = (double *)calloc(c->n[2], sizeof(double));
    c->tau = (double *)calloc(c->n[2], sizeof(double));
    c->work = NULL;
    return c;
}

void or_destroy(void *p)
{
    or_ctx *c = (or_ctx *)p;
    if (!c) return;
    free(c->xe); free(c->ye); free(c->ze);
    free(c->intma); free(c->M);
    free(c->lx); free(c->ly); free(c->lz);
    free(c->rho0); free(c->theta0); free(c->p0); free(c->tau);
    for (int f = 0; f < NF; ++f) { free(c->frc[f].t); free(c->frc[f].vals); }
    free(c->work);
    free(c);
}

void or_sizes(void *p, int64_t *out)
{
    or_ctx *c = (or_ctx *)p;
    out[0] = c->n[0]; out[1] = c->n[1]; out[2] = c->n[2];
    out[3] = c->U; out[4] = c->L; out[5] = c->E;
}

void or_basis(void *p, double *xi, double *w, double *D)
{
    or_ctx *c = (or_ctx *)p;
    memcpy(xi, c->xi, sizeof(double) * c->n1);
    memcpy(w, c->w, sizeof(double) * c->n1);
    memcpy(D, c->D, sizeof(double) * c->n1 * c->n1);
}

void or_lattice_coords(void *p, double *x, double *y, double *z)
{
    or_ctx *c = (or_ctx *)p;
    memcpy(x, c->lx, sizeof(double) * c->n[0]);
    memcpy(y, c->ly, sizeof(double) * c->n[1]);
    memcpy(z, c->lz, sizeof(double) * c->n[2]);
}

void or_mass(void *p, double *M) { or_ctx *c = (or_ctx *)p; memcpy(M, c->M, sizeof(double) * c->U); }
void or_intma(void *p, int64_t *im) { or_ctx *c = (or_ctx *)p; memcpy(im, c->intma, sizeof(int64_t) * c->L); }

/* Rayleigh sponge profile, reading: tau(z) = tau_max sin^2(pi/2 (z - z_s)/(H - z_s))
   above z_s, zero below; applied to u, v, w, theta' (not rho'). */
static double sponge_tau(double z, double zs, double H, double taumax)
{
    if (taumax <= 0.0 || z < zs || H <= zs) return 0.0;
    double s = sin(0.5 * M_PI * (z - zs) / (H - zs));
    return taumax * s * s;
}

void or_set_physics(void *p, double g, double R, double cp, double cv, double pa,
                    double fcor, double zs, double taumax)
{
    or_ctx *c = (or_ctx *)p;
    c->g = g; c->R = R; c->cp = cp; c->cv = cv; c->pa = pa;
    c->fcor = fcor; c->zs = zs; c->taumax = taumax;
    double H = c->ze[c->nel[2]];
    for (int k = 0; k < c->n[2]; ++k) c->tau[k] = sponge_tau(c->lz[k], zs, H, taumax);
}

/* Equation of state (Sec. 2.1): p = p_a (rho R theta / p_a)^gamma. */
static double eos(const or_ctx *c, double rho, double theta)
{
    return c->pa * pow(rho * c->R * theta / c->pa, c->cp / c->cv);
}

/* Reference state per level; p0 := EOS(rho0, theta0) so that a resting
   reference has p' = 0 exactly. */
void or_set_reference(void *p, const double *rho0, const double *theta0)
{
    or_ctx *c = (or_ctx *)p;
    for (int k = 0; k < c->n[2]; ++k) {
        c->rho0[k] = rho0[k];
        c->theta0[k] = theta0[k];
        c->p0[k] = eos(c, rho0[k], theta0[k]);
    }
}

void or_reference_pressure(void *p, double *p0)
{
    or_ctx *c = (or_ctx *)p;
    memcpy(p0, c->p0, sizeof(double) * c->n[2]);
}

/* Prescribed forcing added to the tendency of one field (the heating source
   S_theta of Eq. governing:theta for field 4; any field for manufactured
   solutions).  Values at nsnap times are linearly interpolated in time and
   held constant outside [t_0, t_last] (reading of the 11-sample heating). */
int or_set_forcing(void *p, int field, int nsnap, const double *t, const double *vals)
{
    or_ctx *c = (or_ctx *)p;
    if (field < 0 || field >= NF) return -1;
    forcing_t *f = &c->frc[field];
    free(f->t); free(f->vals);
    f->t = NULL; f->vals = NULL; f->nsnap = 0;
    if (nsnap <= 0) return 0;
    f->nsnap = nsnap;
    f->t = (double *)malloc(sizeof(double) * nsnap);
    f->vals = (double *)malloc(sizeof(double) * nsnap * c->U);
    memcpy(f->t, t, sizeof(double) * nsnap);
    memcpy(f->vals, vals, sizeof(double) * nsnap * c->U);
    return 0;
}

static double forcing_at(const forcing_t *f, int64_t U, int64_t I, double t)
{
    if (f->nsnap == 0) return 0.0;
    if (f->nsnap == 1 || t <= f->t[0]) return f->vals[I];
    if (t >= f->t[f->nsnap - 1]) return f->vals[(int64_t)(f->nsnap - 1) * U + I];
    int k = 0;
    while (k + 1 < f->nsnap - 1 && t >= f->t[k + 1]) ++k;
    double lam = (t - f->t[k]) / (f->t[k + 1] - f->t[k]);
    return (1.0 - lam) * f->vals[(int64_t)k * U + I] + lam * f->vals[(int64_t)(k + 1) * U + I];
}

/*
 * Perturbation pressure p' = EOS(rho0+rho', theta0+theta') - p0.
 * Reading: evaluated through the exact identity
 *     p/p0 = ((1 + rho'/rho0)(1 + theta'/theta0))^gamma
 * as p' = p0 expm1(gamma log1p(s)),  s = a + b + a b,  a = rho'/rho0,
 * b = theta'/theta0, which avoids the cancellation of subtracting two
 * ~1e5 Pa numbers; a resting state gives p' = 0 exactly.
 */
static double pprime(const or_ctx *c, int lev, double rhop, double thetap)
{
    double a = rhop / c->rho0[lev];
    double b = thetap / c->theta0[lev];
    double s = (a + b) + a * b;
    return c->p0[lev] * expm1((c->cp / c->cv) * log1p(s));
}

/*
 * Element tendencies r(f, e, k, j, i) = w_i w_j w_k J^e S_f at every local
 * node (Algorithm 1: gather, gradient, divergence, evaluate f(grad q)).
 * S (Eq. governing, hyper-diffusion excluded):
 *   S_rho'   = - div(rho u)                                 rho = rho0 + rho'
 *   S_u      = - u.grad u - (1/rho) dp'/dx + f v - tau u
 *   S_v      = - u.grad v - (1/rho) dp'/dy - f u - tau v
 *   S_w      = - u.grad w - (1/rho) dp'/dz - (rho'/rho) g - tau w
 *   S_theta' = - u.grad(theta0 + theta') + Q - tau theta'
 * Coriolis (f-plane) and the Rayleigh sponge are the workload's additions;
 * Q is the prescribed forcing.  Derivatives are reference-space contractions
 * with D (Algorithm 2) scaled by the affine metric 2/h.
 */
/* Tendency r[f][m] = w_i w_j w_k J^e S_f of one element e at its (N+1)^3
   local nodes m = i + (N+1)(j + (N+1) k). */
static void element_one(const or_ctx *c, int64_t e, double t, const double *q, double *r, int64_t rstride)
{
    const int n1 = c->n1, np = c->np;
    const int64_t U = c->U;
    const int nxy = c->n[0] * c->n[1];
    double F[8][MAXNP];      /* p', u, v, w, theta, rho u, rho v, rho w */
    double rhoL[MAXNP], rpL[MAXNP], tpL[MAXNP];
    int ex = (int)(e % c->nel[0]), ey = (int)((e / c->nel[0]) % c->nel[1]);
    int ez = (int)(e / ((int64_t)c->nel[0] * c->nel[1]));
    double hx = c->xe[ex + 1] - c->xe[ex], hy = c->ye[ey + 1] - c->ye[ey], hz = c->ze[ez + 1] - c->ze[ez];
    double J = hx * hy * hz / 8.0;
    /* global -> local gather and pointwise derived quantities */
    for (int m = 0; m < np; ++m) {
        int64_t I = c->intma[e * np + m];
        int lev = (int)(I / nxy);
        double rp = q[0 * U + I], u = q[1 * U + I], v = q[2 * U + I], w = q[3 * U + I], tp = q[4 * U + I];
        double rho = c->rho0[lev] + rp;
        F[0][m] = pprime(c, lev, rp, tp);
        F[1][m] = u;
        F[2][m] = v;
        F[3][m] = w;
        F[4][m] = c->theta0[lev] + tp;
        F[5][m] = rho * u;
        F[6][m] = rho * v;
        F[7][m] = rho * w;
        rhoL[m] = rho;
        rpL[m] = rp;
        tpL[m] = tp;
    }
    for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                int m = i + n1 * (j + n1 * k);
                /* reference derivatives (Algorithm 2) */
                double dxi[8], deta[8], dzeta[8];
                for (int f = 0; f < 8; ++f) {
                    double a = 0.0, b = 0.0, cc = 0.0;
                    for (int l = 0; l < n1; ++l) {
                        a += c->D[i * n1 + l] * F[f][l + n1 * (j + n1 * k)];
                        b += c->D[j * n1 + l] * F[f][i + n1 * (l + n1 * k)];
                        cc += c->D[k * n1 + l] * F[f][i + n1 * (j + n1 * l)];
                    }
                    dxi[f] = a; deta[f] = b; dzeta[f] = cc;
                }
                /* metric terms of the affine map */
                double mx = 2.0 / hx, my = 2.0 / hy, mz = 2.0 / hz;
                double gx[5], gy[5], gz[5];
                for (int f = 0; f < 5; ++f) { gx[f] = mx * dxi[f]; gy[f] = my * deta[f]; gz[f] = mz * dzeta[f]; }
                double divm = mx * dxi[5] + my * deta[6] + mz * dzeta[7];
                int64_t I = c->intma[e * np + m];
                int lev = (int)(I / nxy);
                double u = F[1][m], v = F[2][m], w = F[3][m];
                double rho = rhoL[m];
                double tau = c->tau[lev];
                double S[5];
                S[0] = -divm;
                S[1] = -(u * gx[1] + v * gy[1] + w * gz[1]) - gx[0] / rho + c->fcor * v - tau * u;
                S[2] = -(u * gx[2] + v * gy[2] + w * gz[2]) - gy[0] / rho - c->fcor * u - tau * v;
                S[3] = -(u * gx[3] + v * gy[3] + w * gz[3]) - gz[0] / rho - (rpL[m] / rho) * c->g - tau * w;
                S[4] = -(u * gx[4] + v * gy[4] + w * gz[4]) - tau * tpL[m];
                for (int f = 0; f < 5; ++f) S[f] += forcing_at(&c->frc[f], U, I, t);
                double wJ = c->w[i] * c->w[j] * c->w[k] * J;
                for (int f = 0; f < 5; ++f) r[f * rstride + m] = wJ * S[f];
            }
}

/*
 * Element tendencies r(f, e, k, j, i) = w_i w_j w_k J^e S_f at every local
 * node (Algorithm 1: gather, gradient, divergence, evaluate f(grad q)).
 * S (Eq. governing, hyper-diffusion excluded):
 *   S_rho'   = - div(rho u)                                 rho = rho0 + rho'
 *   S_u      = - u.grad u - (1/rho) dp'/dx + f v - tau u
 *   S_v      = - u.grad v - (1/rho) dp'/dy - f u - tau v
 *   S_w      = - u.grad w - (1/rho) dp'/dz - (rho'/rho) g - tau w
 *   S_theta' = - u.grad(theta0 + theta') + Q - tau theta'
 * Coriolis (f-plane) and the Rayleigh sponge are the workload's additions;
 * Q is the prescribed forcing.  Derivatives are reference-space contractions
 * with D (Algorithm 2) scaled by the affine metric 2/h.
 */
void or_element_tendency(void *p, double t, const double *q, double *r)
{
    or_ctx *c = (or_ctx *)p;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < c->E; ++e) element_one(c, e, t, q, r + e * c->np, c->L);
}

/* The right-hand side at a sample of unique nodes only: the same element
   tendencies, DSS (ascending element order) and mass inverse as or_rhs,
   restricted to the elements that contain a requested node.  out is
   [5][n]; nodes must be distinct unique-node indices I (returns -1, and
   computes nothing, on a repeated or out-of-range index). */
int or_rhs_sample(void *p, double t, const double *q, int64_t n, const int64_t *nodes, double *out)
{
    or_ctx *c = (or_ctx *)p;
    const int np = c->np;
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * c->U);
    for (int64_t I = 0; I < c->U; ++I) slot[I] = -1;
    for (int64_t s = 0; s < n; ++s) {
        if (nodes[s] < 0 || nodes[s] >= c->U || slot[nodes[s]] >= 0) {
            free(slot);
            return -1;
        }
        slot[nodes[s]] = s;
    }
    for (int64_t s = 0; s < 5 * n; ++s) out[s] = 0.0;
    double r[5 * MAXNP];
    for (int64_t e = 0; e < c->E; ++e) {
        int hit = 0;
        for (int m = 0; m < np && !hit; ++m) hit = slot[c->intma[e * np + m]] >= 0;
        if (!hit) continue;
        element_one(c, e, t, q, r, np);
        for (int m = 0; m < np; ++m) {
            int64_t s = slot[c->intma[e * np + m]];
            if (s < 0) continue;
            for (int f = 0; f < NF; ++f) out[f * n + s] += r[f * np + m];
        }
    }
    const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
    for (int64_t s = 0; s < n; ++s) {
        int64_t I = nodes[s];
        for (int f = 0; f < NF; ++f) out[f * n + s] /= c->M[I];
        int ix = (int)(I % nx), iy = (int)((I / nx) % ny), iz = (int)(I / ((int64_t)nx * ny));
        if (!c->per[0] && (ix == 0 || ix == nx - 1)) out[1 * n + s] = 0.0;
        if (!c->per[1] && (iy == 0 || iy == ny - 1)) out[2 * n + s] = 0.0;
        if (iz == 0 || iz == nz - 1) out[3 * n + s] = 0.0;
    }
    free(slot);
    return 0;
}

/* Zero the wall-normal velocity tendency at no-flux boundaries (reading:
   strong enforcement after DSS; x/y walls only when not periodic, z = 0 and
   z = H always). */
static void apply_walls(const or_ctx *c, double *dq)
{
    const int64_t U = c->U;
    const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
    for (int64_t I = 0; I < U; ++I) {
        int ix = (int)(I % nx), iy = (int)((I / nx) % ny), iz = (int)(I / ((int64_t)nx * ny));
        if (!c->per[0] && (ix == 0 || ix == nx - 1)) dq[1 * U + I] = 0.0;
        if (!c->per[1] && (iy == 0 || iy == ny - 1)) dq[2 * U + I] = 0.0;
        if (iz == 0 || iz == nz - 1) dq[3 * U + I] = 0.0;
    }
}

/* DSS gather (Algorithm 3): out_I = sum over (e, local) -> I of in, summed in
   ascending (e, k, j, i) order.  mode 0: plain sum; mode 1: sum of
   w_i w_j w_k J^e * in, divided by M_I (mass-weighted average). */
void or_dss(void *p, int nfields, int mode, const double *E, double *out)
{
    or_ctx *c = (or_ctx *)p;
    const int n1 = c->n1, np = c->np;
    for (int f = 0; f < nfields; ++f) {
        double *o = out + (int64_t)f * c->U;
        const double *in = E + (int64_t)f * c->L;
        for (int64_t I = 0; I < c->U; ++I) o[I] = 0.0;
        for (int64_t e = 0; e < c->E; ++e) {
            double J = 1.0;
            if (mode == 1) {
                int ex = (int)(e % c->nel[0]), ey = (int)((e / c->nel[0]) % c->nel[1]);
                int ez = (int)(e / ((int64_t)c->nel[0] * c->nel[1]));
                J = (c->xe[ex + 1] - c->xe[ex]) * (c->ye[ey + 1] - c->ye[ey]) * (c->ze[ez + 1] - c->ze[ez]) / 8.0;
            }
            for (int k = 0; k < n1; ++k)
                for (int j = 0; j < n1; ++j)
                    for (int i = 0; i < n1; ++i) {
                        int m = i + n1 * (j + n1 * k);
                        double v = in[e * np + m];
                        if (mode == 1) v = c->w[i] * c->w[j] * c->w[k] * J * v;
                        o[c->intma[e * np + m]] += v;
                    }
        }
        if (mode == 1)
            for (int64_t I = 0; I < c->U; ++I) o[I] /= c->M[I];
    }
}

/* Global-to-local scatter (Algorithm 1 gather / Algorithm 3 scatter):
   E(f, e, local) = U(f, intma(e, local)). */
void or_scatter(void *p, int nfields, const double *Uin, double *E)
{
    or_ctx *c = (or_ctx *)p;
    for (int f = 0; f < nfields; ++f)
        for (int64_t m = 0; m < c->L; ++m)
            E[(int64_t)f * c->L + m] = Uin[(int64_t)f * c->U + c->intma[m]];
}

/* dq/dt = M^{-1} DSS(w J S) with wall conditions (Eq. governing:matrix). */
void or_rhs(void *p, double t, const double *q, double *dq)
{
    or_ctx *c = (or_ctx *)p;
    if (!c->work) c->work = (double *)malloc(sizeof(double) * NF * c->L);
    or_element_tendency(p, t, q, c->work);
    const int64_t U = c->U, L = c->L;
    for (int f = 0; f < NF; ++f) {
        double *o = dq + f * U;
        for (int64_t I = 0; I < U; ++I) o[I] = 0.0;
        for (int64_t m = 0; m < L; ++m) o[c->intma[m]] += c->work[f * L + m];
        for (int64_t I = 0; I < U; ++I) o[I] /= c->M[I];
    }
    apply_walls(c, dq);
}

/* Three-stage third-order SSP Runge-Kutta:
     q1 = q^n + dt R(q^n, t)
     q2 = 3/4 q^n + 1/4 (q1 + dt R(q1, t + dt))
     q^{n+1} = 1/3 q^n + 2/3 (q2 + dt R(q2, t + dt/2))          */
void or_rk3(void *p, double t, double dt, int nsteps, double *q)
{
    or_ctx *c = (or_ctx *)p;
    const int64_t n = NF * c->U;
    double *q1 = (double *)malloc(sizeof(double) * n);
    double *q2 = (double *)malloc(sizeof(double) * n);
    double *R = (double *)malloc(sizeof(double) * n);
    for (int s = 0; s < nsteps; ++s) {
        double ts = t + s * dt;
        or_rhs(p, ts, q, R);
        for (int64_t i = 0; i < n; ++i) q1[i] = q[i] + dt * R[i];
        or_rhs(p, ts + dt, q1, R);
        for (int64_t i = 0; i < n; ++i) q2[i] = 0.75 * q[i] + 0.25 * (q1[i] + dt * R[i]);
        or_rhs(p, ts + 0.5 * dt, q2, R);
        for (int64_t i = 0; i < n; ++i) q[i] = q[i] / 3.0 + (2.0 / 3.0) * (q2[i] + dt * R[i]);
    }
    free(q1); free(q2); free(R);
}

/*
 * Vertical linear operator of the 1D-IMEX (HEVI) split (Sec. 2.3): the
 * linearisation of S about the resting reference restricted to vertical
 * derivatives, with p'_L = gamma p0 (rho'/rho0 + theta'/theta0):
 *   (L_v)_rho'   = - d/dz (rho0 w)
 *   (L_v)_w      = - (1/rho0) dp'_L/dz - g rho'/rho0
 *   (L_v)_theta' = - w dtheta0/dz
 *   (L_v)_u = (L_v)_v = 0.
 * Discretised like S: element-local contractions along z weighted by
 * w_i w_j w_k J^e, DSS, divided by M, w-row zero at z = 0 and z = H.
 * Applied to a full [5][U] vector.
 */
void or_lv_apply(void *p, const double *x, double *y)
{
    or_ctx *c = (or_ctx *)p;
    const int N = c->N, n1 = c->n1, np = c->np;
    const int64_t U = c->U, L = c->L;
    const double gam = c->cp / c->cv;
    const int nxy = c->n[0] * c->n[1];
    if (!c->work) c->work = (double *)malloc(sizeof(double) * NF * c->L);
    double *r = c->work;
    (void)N;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < c->E; ++e) {
        double F[3][MAXNP];  /* rho0 w, p'_L, theta0 */
        int ex = (int)(e % c->nel[0]), ey = (int)((e / c->nel[0]) % c->nel[1]);
        int ez = (int)(e / ((int64_t)c->nel[0] * c->nel[1]));
        double hx = c->xe[ex + 1] - c->xe[ex], hy = c->ye[ey + 1] - c->ye[ey], hz = c->ze[ez + 1] - c->ze[ez];
        double J = hx * hy * hz / 8.0;
        for (int m = 0; m < np; ++m) {
            int64_t I = c->intma[e * np + m];
            int lev = (int)(I / nxy);
            F[0][m] = c->rho0[lev] * x[3 * U + I];
            F[1][m] = gam * c->p0[lev] * (x[0 * U + I] / c->rho0[lev] + x[4 * U + I] / c->theta0[lev]);
            F[2][m] = c->theta0[lev];
        }
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    int m = i + n1 * (j + n1 * k);
                    double d[3] = {0.0, 0.0, 0.0};
                    for (int f = 0; f < 3; ++f)
                        for (int l = 0; l < n1; ++l)
                            d[f] += c->D[k * n1 + l] * F[f][i + n1 * (j + n1 * l)];
                    double mz = 2.0 / hz;
                    int64_t I = c->intma[e * np + m];
                    int lev = (int)(I / nxy);
                    double S[5];
                    S[0] = -mz * d[0];
                    S[1] = 0.0;
                    S[2] = 0.0;
                    S[3] = -mz * d[1] / c->rho0[lev] - c->g * x[0 * U + I] / c->rho0[lev];
                    S[4] = -x[3 * U + I] * mz * d[2];
                    double wJ = c->w[i] * c->w[j] * c->w[k] * J;
                    for (int f = 0; f < 5; ++f) r[f * L + e * np + m] = wJ * S[f];
                }
    }
    for (int f = 0; f < NF; ++f) {
        double *o = y + f * U;
        for (int64_t I = 0; I < U; ++I) o[I] = 0.0;
        for (int64_t m = 0; m < L; ++m) o[c->intma[m]] += r[f * L + m];
        for (int64_t I = 0; I < U; ++I) o[I] /= c->M[I];
    }
    for (int64_t I = 0; I < U; ++I) {
        int iz = (int)(I / nxy);
        if (iz == 0 || iz == c->n[2] - 1) y[3 * U + I] = 0.0;
    }
}

/*
 * Linear operator of the 3D-IMEX split (Sec. 2.3): the linearisation of S
 * about the resting reference in all three directions (acoustic and gravity
 * terms), with p'_L = gamma p0 (rho'/rho0 + theta'/theta0), plus the
 * implicit upper absorbing layer of the w equation (damping -tau(z) w, the
 * Klemp form; the Rayleigh damping of u, v and theta' stays explicit):
 *   (L)_rho'   = - d/dx (rho0 u) - d/dy (rho0 v) - d/dz (rho0 w)
 *   (L)_u      = - (1/rho0) dp'_L/dx
 *   (L)_v      = - (1/rho0) dp'_L/dy
 *   (L)_w      = - (1/rho0) dp'_L/dz - g rho'/rho0 - tau w
 *   (L)_theta' = - w dtheta0/dz.
 * Discretised like S (element-local contractions weighted by w_i w_j w_k J,
 * DSS, divided by M) with the wall conditions of S.
 */
void or_l3_apply(void *p, const double *x, double *y)
{
    or_ctx *c = (or_ctx *)p;
    const int n1 = c->n1, np = c->np;
    const int64_t U = c->U, L = c->L;
    const double gam = c->cp / c->cv;
    const int nxy = c->n[0] * c->n[1];
    if (!c->work) c->work = (double *)malloc(sizeof(double) * NF * c->L);
    double *r = c->work;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < c->E; ++e) {
        double F[5][MAXNP];  /* rho0 u, rho0 v, rho0 w, p'_L, theta0 */
        int ex = (int)(e % c->nel[0]), ey = (int)((e / c->nel[0]) % c->nel[1]);
        int ez = (int)(e / ((int64_t)c->nel[0] * c->nel[1]));
        double hx = c->xe[ex + 1] - c->xe[ex], hy = c->ye[ey + 1] - c->ye[ey], hz = c->ze[ez + 1] - c->ze[ez];
        double J = hx * hy * hz / 8.0;
        for (int m = 0; m < np; ++m) {
            int64_t I = c->intma[e * np + m];
            int lev = (int)(I / nxy);
            F[0][m] = c->rho0[lev] * x[1 * U + I];
            F[1][m] = c->rho0[lev] * x[2 * U + I];
            F[2][m] = c->rho0[lev] * x[3 * U + I];
            F[3][m] = gam * c->p0[lev] * (x[0 * U + I] / c->rho0[lev] + x[4 * U + I] / c->theta0[lev]);
            F[4][m] = c->theta0[lev];
        }
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    int m = i + n1 * (j + n1 * k);
                    double dx0 = 0.0, dy1 = 0.0, dz2 = 0.0, dxp = 0.0, dyp = 0.0, dzp = 0.0, dzt = 0.0;
                    for (int l = 0; l < n1; ++l) {
                        int mx = l + n1 * (j + n1 * k), my = i + n1 * (l + n1 * k), mz = i + n1 * (j + n1 * l);
                        dx0 += c->D[i * n1 + l] * F[0][mx];
                        dxp += c->D[i * n1 + l] * F[3][mx];
                        dy1 += c->D[j * n1 + l] * F[1][my];
                        dyp += c->D[j * n1 + l] * F[3][my];
                        dz2 += c->D[k * n1 + l] * F[2][mz];
                        dzp += c->D[k * n1 + l] * F[3][mz];
                        dzt += c->D[k * n1 + l] * F[4][mz];
                    }
                    double ax = 2.0 / hx, ay = 2.0 / hy, az = 2.0 / hz;
                    int64_t I = c->intma[e * np + m];
                    int lev = (int)(I / nxy);
                    double S[5];
                    S[0] = -(ax * dx0 + ay * dy1 + az * dz2);
                    S[1] = -ax * dxp / c->rho0[lev];
                    S[2] = -ay * dyp / c->rho0[lev];
                    S[3] = -az * dzp / c->rho0[lev] - c->g * x[0 * U + I] / c->rho0[lev] - c->tau[lev] * x[3 * U + I];
                    S[4] = -x[3 * U + I] * az * dzt;
                    double wJ = c->w[i] * c->w[j] * c->w[k] * J;
                    for (int f = 0; f < 5; ++f) r[f * L + e * np + m] = wJ * S[f];
                }
    }
    for (int f = 0; f < NF; ++f) {
        double *o = y + f * U;
        for (int64_t I = 0; I < U; ++I) o[I] = 0.0;
        for (int64_t m = 0; m < L; ++m) o[c->intma[m]] += r[f * L + m];
        for (int64_t I = 0; I < U; ++I) o[I] /= c->M[I];
    }
    apply_walls(c, y);
}

/* Threads an OpenMP loop of the oracle uses. */
int or_num_threads(void) { return omp_get_max_threads(); }

/* Sets the threads of the oracle's later parallel loops (n >= 1). */
void or_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
