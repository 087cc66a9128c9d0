/*
 * lbm_oracle.c -- plain FP64 CPU oracle of the coupled central-moment LB step
 * (arXiv 2408.00146).  TEST INFRASTRUCTURE ONLY: it checks the GPU library and
 * must never be part of the product path.
 *
 * The step follows the paper's algorithm literally: for each of the four
 * distribution sets, raw moments by the matrix P, central moments by the
 * matrix F(u), relaxation of each central moment to its equilibrium, back
 * through F^-1(u) and P^-1 (all dense 9x9 products, App. F), then streaming.
 * Coupling fields (gradients, curvature, surface tension, forces) are formed
 * from the zeroth moments exactly as stated in Sec. 2 and Sec. 3.  Where the
 * text is garbled or silent the reading taken is stated next to the code.
 *
 * Built with -O2 -ffp-contract=off -fno-fast-math; OpenMP over rows only.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- lattice */
/* D2Q9 velocity set of App. B.  The printed x-list ends in 0; the ninth
 * velocity is (1,-1), as the second row of the printed P matrix has it. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double WT[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

static char g_err[256];
const char* orc_error(void) { return g_err; }

/* ------------------------------------------------------ App. F matrices */
/* P: distributions -> raw moments (00,10,01,20,02,11,21,12,22), as printed. */
static const double PMAT[81] = {
    1, 1, 1, 1, 1, 1, 1, 1, 1,
    0, 1, 0, -1, 0, 1, -1, -1, 1,
    0, 0, 1, 0, -1, 1, 1, -1, -1,
    0, 1, 0, 1, 0, 1, 1, 1, 1,
    0, 0, 1, 0, 1, 1, 1, 1, 1,
    0, 0, 0, 0, 0, 1, -1, 1, -1,
    0, 0, 0, 0, 0, 1, 1, -1, -1,
    0, 0, 0, 0, 0, 1, -1, -1, 1,
    0, 0, 0, 0, 0, 1, 1, 1, 1};

/* P^-1: raw moments -> distributions, as printed. */
static const double PINV[81] = {
    1, 0, 0, -1, -1, 0, 0, 0, 1,
    0, 0.5, 0, 0.5, 0, 0, 0, -0.5, -0.5,
    0, 0, 0.5, 0, 0.5, 0, -0.5, 0, -0.5,
    0, -0.5, 0, 0.5, 0, 0, 0, 0.5, -0.5,
    0, 0, -0.5, 0, 0.5, 0, 0.5, 0, -0.5,
    0, 0, 0, 0, 0, 0.25, 0.25, 0.25, 0.25,
    0, 0, 0, 0, 0, -0.25, 0.25, -0.25, 0.25,
    0, 0, 0, 0, 0, 0.25, -0.25, -0.25, 0.25,
    0, 0, 0, 0, 0, -0.25, -0.25, 0.25, 0.25};

void orc_matrix_P(double out[81]) { memcpy(out, PMAT, sizeof PMAT); }
void orc_matrix_Pinv(double out[81]) { memcpy(out, PINV, sizeof PINV); }

/* F(u): raw -> central moments, rows as printed in App. F.  Reading: in the
 * last row the coefficients of the raw moments 10 and 01 are -2 ux uy^2 and
 * -2 ux^2 uy (binomial expansion of (ex-ux)^2 (ey-uy)^2, which the text says
 * F follows); the printed -ux uy^2, -ux^2 uy break F(u) F(-u) = I. */
void orc_matrix_F(double ux, double uy, double F[81])
{
    const double x2 = ux * ux, y2 = uy * uy;
    const double rows[81] = {
        1, 0, 0, 0, 0, 0, 0, 0, 0,
        -ux, 1, 0, 0, 0, 0, 0, 0, 0,
        -uy, 0, 1, 0, 0, 0, 0, 0, 0,
        x2, -2 * ux, 0, 1, 0, 0, 0, 0, 0,
        y2, 0, -2 * uy, 0, 1, 0, 0, 0, 0,
        ux * uy, -uy, -ux, 0, 0, 1, 0, 0, 0,
        -x2 * uy, 2 * ux * uy, x2, -uy, 0, -2 * ux, 1, 0, 0,
        -ux * y2, y2, 2 * ux * uy, 0, -ux, -2 * uy, 0, 1, 0,
        x2 * y2, -2 * ux * y2, -2 * x2 * uy, y2, x2, 4 * ux * uy, -2 * uy, -2 * ux, 1};
    memcpy(F, rows, sizeof rows);
}

/* F^-1(u): central -> raw moments, rows as printed (same last-row reading). */
void orc_matrix_Finv(double ux, double uy, double F[81])
{
    const double x2 = ux * ux, y2 = uy * uy;
    const double rows[81] = {
        1, 0, 0, 0, 0, 0, 0, 0, 0,
        ux, 1, 0, 0, 0, 0, 0, 0, 0,
        uy, 0, 1, 0, 0, 0, 0, 0, 0,
        x2, 2 * ux, 0, 1, 0, 0, 0, 0, 0,
        y2, 0, 2 * uy, 0, 1, 0, 0, 0, 0,
        ux * uy, uy, ux, 0, 0, 1, 0, 0, 0,
        x2 * uy, 2 * ux * uy, x2, uy, 0, 2 * ux, 1, 0, 0,
        ux * y2, y2, 2 * ux * uy, 0, ux, 2 * uy, 0, 1, 0,
        x2 * y2, 2 * ux * y2, 2 * x2 * uy, y2, x2, 4 * ux * uy, 2 * uy, 2 * ux, 1};
    memcpy(F, rows, sizeof rows);
}

static void matvec9(const double M[81], const double v[9], double out[9])
{
    for (int r = 0; r < 9; ++r) {
        double acc = 0.0;
        for (int c = 0; c < 9; ++c) acc += M[r * 9 + c] * v[c];
        out[r] = acc;
    }
}

/* distribution -> central moments: kappa = F(u) P x */
static void to_central(const double x[9], double ux, double uy, double kap[9])
{
    double raw[9], F[81];
    matvec9(PMAT, x, raw);
    orc_matrix_F(ux, uy, F);
    matvec9(F, raw, kap);
}

/* central moments -> distribution: x = P^-1 F^-1(u) kappa */
static void from_central(const double kap[9], double ux, double uy, double x[9])
{
    double raw[9], Fi[81];
    orc_matrix_Finv(ux, uy, Fi);
    matvec9(Fi, kap, raw);
    matvec9(PINV, raw, x);
}

/* ------------------------------------------- advection-diffusion collision */
/* Shared by f (App. B), h (App. D) and q (App. E): every central moment
 * relaxes to its equilibrium; first-order moments at rate omega1, all others
 * at rate 1.  Equilibrium central moments: (X, jx, jy, cs2 X, cs2 X, 0, 0, 0,
 * cs2^2 X), where (jx, jy) is the set's first-order equilibrium. */
void orc_collide_ad(const double pop[9], double X, double jx, double jy, double omega1,
                    double ux, double uy, double out[9])
{
    double kap[9], eq[9], om[9];
    to_central(pop, ux, uy, kap);
    eq[0] = X;
    eq[1] = jx;
    eq[2] = jy;
    eq[3] = CS2 * X;
    eq[4] = CS2 * X;
    eq[5] = 0.0;
    eq[6] = 0.0;
    eq[7] = 0.0;
    eq[8] = CS2 * CS2 * X;
    for (int k = 0; k < 9; ++k) om[k] = 1.0;
    om[1] = omega1;
    om[2] = omega1;
    double post[9];
    for (int k = 0; k < 9; ++k) post[k] = kap[k] + om[k] * (eq[k] - kap[k]);
    from_central(post, ux, uy, out);
}

/* ------------------------------------------------- two-fluid collision */
/* Equilibrium central moments of the pressure-based scheme (App. C), with
 * varphi = p - rho cs2.  The 22 moment, printed as
 * cs2^3 rho + varphi (ux^2 + cs2)(uy^2 + cs2), is evaluated in the equal form
 * p cs2^2 + varphi (cs2 (ux^2 + uy^2) + ux^2 uy^2): the printed one cancels two
 * O(rho/27) terms down to O(p/9) and loses ~12 digits of p. */
void orc_eq_g(double p, double rho, double ux, double uy, double eq[9])
{
    const double vp = p - rho * CS2;
    eq[0] = p;
    eq[1] = -vp * ux;
    eq[2] = -vp * uy;
    eq[3] = p * CS2 + vp * ux * ux;
    eq[4] = p * CS2 + vp * uy * uy;
    eq[5] = vp * ux * uy;
    eq[6] = -vp * (ux * ux + CS2) * uy;
    eq[7] = -vp * (uy * uy + CS2) * ux;
    eq[8] = p * CS2 * CS2 + vp * (CS2 * (ux * ux + uy * uy) + ux * ux * uy * uy);
}

/* Central moments of the source (App. C); Gamma00 = Fp . u.  Third- and
 * fourth-order source moments are zero as the paper sets them. */
void orc_source_g(double Ftx, double Fty, double Fpx, double Fpy, double ux, double uy, double s[9])
{
    const double G = Fpx * ux + Fpy * uy;
    s[0] = G;
    s[1] = CS2 * Ftx - ux * G;
    s[2] = CS2 * Fty - uy * G;
    s[3] = 2.0 * CS2 * Fpx * ux + (ux * ux + CS2) * G;
    s[4] = 2.0 * CS2 * Fpy * uy + (uy * uy + CS2) * G;
    s[5] = CS2 * (Fpx * uy + Fpy * ux) + ux * uy * G;
    s[6] = 0.0;
    s[7] = 0.0;
    s[8] = 0.0;
}

/* Collision of g (App. C): the diagonal second-order moments are regrouped
 * into trace (2s) and deviator (2d); each moment takes
 *     eta~ = eta + w (eta_eq - eta) + (1 - w/2) sigma,
 * with w_2d = w_11 = omega_nu (shear viscosity) and all other rates 1
 * (bulk viscosity from w_2s = 1); then 20/02 are recovered from 2s/2d. */
void orc_collide_g(const double g[9], double p, double rho, double ux, double uy,
                   double Ftx, double Fty, double Fpx, double Fpy, double omega_nu, double out[9])
{
    double eta[9], eq[9], src[9];
    to_central(g, ux, uy, eta);
    orc_eq_g(p, rho, ux, uy, eq);
    orc_source_g(Ftx, Fty, Fpx, Fpy, ux, uy, src);

    /* basis (00, 10, 01, 2s, 2d, 11, 21, 12, 22) */
    double b[9], beq[9], bs[9], om[9];
    for (int k = 0; k < 9; ++k) {
        b[k] = eta[k];
        beq[k] = eq[k];
        bs[k] = src[k];
        om[k] = 1.0;
    }
    b[3] = eta[3] + eta[4];
    b[4] = eta[3] - eta[4];
    beq[3] = eq[3] + eq[4];
    beq[4] = eq[3] - eq[4];
    bs[3] = src[3] + src[4];
    bs[4] = src[3] - src[4];
    om[4] = omega_nu; /* 2d */
    om[5] = omega_nu; /* 11 */

    double post[9];
    for (int k = 0; k < 9; ++k) post[k] = b[k] + om[k] * (beq[k] - b[k]) + (1.0 - 0.5 * om[k]) * bs[k];
    const double t2s = post[3], t2d = post[4];
    post[3] = 0.5 * (t2s + t2d);
    post[4] = 0.5 * (t2s - t2d);
    from_central(post, ux, uy, out);
}

/* ------------------------------------------------------------- state */
#define GH 2 /* ghost frame width of the work fields */

struct orc_state {
    orc_case c;
    int nx, ny, ex; /* ex = nx + 2*GH, row stride of extended fields */
    size_t n, next;
    double* pop;  /* [4][9][n] post-streaming populations */
    double* post; /* [4][9][n] post-collision populations */
    /* domain fields */
    double *phi, *T, *psi, *ps, *jx, *jy;
    /* extended fields (ghost frame GH) */
    double *phiE, *TE, *psiE, *psE, *sigE, *gxE, *gyE, *nxE, *nyE;
    /* per-node results of the macroscopic stage */
    double *rho, *ux, *uy, *p, *kap, *Fsx, *Fsy, *Fpx, *Fpy, *Ftx, *Fty, *Rx, *Ry, *omnu, *omT;
    int64_t step;
};

static size_t eidx(const orc_state* s, int i, int j) { return (size_t)(j + GH) * s->ex + (size_t)(i + GH); }

static double* alloc_d(size_t n)
{
    double* p = (double*)calloc(n, sizeof(double));
    if (!p) {
        fprintf(stderr, "oracle: out of memory\n");
        abort();
    }
    return p;
}

/* ------------------------------------------------------ initial state */
/* splitmix64 (Steele, Lea & Flood 2014): state advances by the golden-ratio
 * increment; output is the state passed through the published mixer. */
static uint64_t splitmix64_nth(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64(uint64_t seed, uint64_t k) { return splitmix64_nth(seed, k); }

/* Uniform in [-1, 1) from the k-th splitmix64 output (53 high bits). */
static double noise_unit(uint64_t seed, uint64_t k)
{
    const uint64_t z = splitmix64_nth(seed, k);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

static double wall_T(const orc_case* c, double x) { return c->T0 + c->gradT * (x - c->xT0); }

/* Clean phase profile of the initial interface: the tanh equilibrium of the
 * conservative Allen-Cahn equation (Sec. 3), phi = 1 inside the bubble. */
static double phi_clean(const orc_case* c, int i, int j)
{
    if (c->init_kind == 2) return 0.0;
    double d;
    if (c->init_kind == 1) {
        d = c->R - fabs((double)j - c->yc);
    } else {
        const double dx = (double)i - c->xc, dy = (double)j - c->yc;
        d = c->R - sqrt(dx * dx + dy * dy);
    }
    return 0.5 + 0.5 * tanh(2.0 * d / c->W);
}

/* Rest equilibrium (u = 0) of all four sets.  For g at u = 0 the central
 * moment equilibria of Sec. 4.2 reduce to those of w_a p (zeroth p, second
 * p c_s^2, fourth p c_s^4), so g_a = w_a p; p = NULL means p = 0. */
static void set_rest_equilibrium(orc_state* s, const double* phi, const double* T, const double* psi,
                                 const double* p)
{
    const size_t n = s->n;
    for (int a = 0; a < 9; ++a) {
        for (size_t k = 0; k < n; ++k) {
            s->pop[(0 * 9 + a) * n + k] = WT[a] * phi[k];
            s->pop[(1 * 9 + a) * n + k] = p ? WT[a] * p[k] : 0.0;
            s->pop[(2 * 9 + a) * n + k] = WT[a] * T[k];
            s->pop[(3 * 9 + a) * n + k] = WT[a] * psi[k];
        }
    }
    s->step = 0;
}

static int validate(const orc_case* c)
{
    if (c->nx < 4 || c->ny < 4) {
        snprintf(g_err, sizeof g_err, "nx, ny must be >= 4");
        return 0;
    }
    if (c->wall[0] != c->wall[1] || c->wall[2] != c->wall[3]) {
        snprintf(g_err, sizeof g_err, "periodic sides must come in pairs");
        return 0;
    }
    if (!(c->W > 0) || !(c->rho_A > 0) || !(c->rho_B > 0) || !(c->nu_A > 0) || !(c->nu_B > 0) ||
        !(c->alpha_A > 0) || !(c->alpha_B > 0) || !(c->D_psi > 0) || !(c->M_phi > 0) || !(c->psi_inf > 0)) {
        snprintf(g_err, sizeof g_err, "W, densities, viscosities, diffusivities, mobility, psi_inf must be > 0");
        return 0;
    }
    return 1;
}

orc_state* orc_create(const orc_case* c)
{
    if (!validate(c)) return NULL;
    orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
    s->c = *c;
    s->nx = c->nx;
    s->ny = c->ny;
    s->ex = c->nx + 2 * GH;
    s->n = (size_t)c->nx * c->ny;
    s->next = (size_t)(c->nx + 2 * GH) * (c->ny + 2 * GH);
    s->pop = alloc_d(36 * s->n);
    s->post = alloc_d(36 * s->n);
    double** dom[] = {&s->phi, &s->T, &s->psi, &s->ps, &s->jx, &s->jy, &s->rho, &s->ux, &s->uy, &s->p,
                      &s->kap, &s->Fsx, &s->Fsy, &s->Fpx, &s->Fpy, &s->Ftx, &s->Fty, &s->Rx, &s->Ry,
                      &s->omnu, &s->omT};
    for (size_t k = 0; k < sizeof dom / sizeof dom[0]; ++k) *dom[k] = alloc_d(s->n);
    double** ext[] = {&s->phiE, &s->TE, &s->psiE, &s->psE, &s->sigE, &s->gxE, &s->gyE, &s->nxE, &s->nyE};
    for (size_t k = 0; k < sizeof ext / sizeof ext[0]; ++k) *ext[k] = alloc_d(s->next);

    /* initial fields */
    double* phi0 = alloc_d(s->n);
    double* T0 = alloc_d(s->n);
    double* psi0 = alloc_d(s->n);
    double* p0 = alloc_d(s->n);
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            const size_t k = (size_t)j * s->nx + i;
            const double pc = phi_clean(c, i, j);
            phi0[k] = pc + c->phi_noise * noise_unit(c->seed, k);
            T0[k] = wall_T(c, (double)i);
            psi0[k] = c->psi_bulk + c->psi_gradx * ((double)i - c->xT0) + c->psi_band * 4.0 * pc * (1.0 - pc);
            /* integral of the CSF weight 1.5 W |grad phi|^2 (Sec. 3) across the
             * tanh profile, |grad phi| = 4 phi (1 - phi) / W: d p / d phi =
             * p_jump 6 phi (1 - phi) */
            p0[k] = c->p_jump * pc * pc * (3.0 - 2.0 * pc);
        }
    set_rest_equilibrium(s, phi0, T0, psi0, p0);
    free(p0);
    free(phi0);
    free(T0);
    free(psi0);
    return s;
}

void orc_free(orc_state* s)
{
    if (!s) return;
    double* all[] = {s->pop, s->post, s->phi, s->T, s->psi, s->ps, s->jx, s->jy, s->rho, s->ux, s->uy,
                     s->p, s->kap, s->Fsx, s->Fsy, s->Fpx, s->Fpy, s->Ftx, s->Fty, s->Rx, s->Ry,
                     s->omnu, s->omT, s->phiE, s->TE, s->psiE, s->psE, s->sigE, s->gxE, s->gyE,
                     s->nxE, s->nyE};
    for (size_t k = 0; k < sizeof all / sizeof all[0]; ++k) free(all[k]);
    free(s);
}

void orc_load_fields(orc_state* s, const double* phi, const double* T, const double* psi)
{
    set_rest_equilibrium(s, phi, T, psi, NULL);
}

int64_t orc_steps_done(const orc_state* s) { return s->step; }

void orc_get_populations(const orc_state* s, double* out) { memcpy(out, s->pop, 36 * s->n * sizeof(double)); }
void orc_set_populations(orc_state* s, const double* in) { memcpy(s->pop, in, 36 * s->n * sizeof(double)); }

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* -------------------------------------------------------- ghost values */
/* Field kinds for the ghost rule. */
enum { GK_MIRROR = 0, GK_TEMP = 1, GK_PSI = 2 };

static int dirichlet_side(const orc_case* c, int kind, int side)
{
    if (kind == GK_TEMP) return c->t_bc[side] == 1;
    if (kind == GK_PSI) return c->psi_bc[side] == 1;
    return 0;
}

static double wall_value(const orc_case* c, int kind, int side, double xw)
{
    if (kind == GK_TEMP) return wall_T(c, xw);
    return c->psi_w[side];
}

/* Value of a domain field X at any node (i, j), in or outside the domain.
 * Reading of the wall treatment for finite differences (the paper does not
 * state it): walls sit halfway between the last fluid node and the first
 * ghost; a ghost takes the value of its mirror node (zero normal gradient),
 * or 2 X_w - X(mirror) on a Dirichlet wall, X_w taken at the wall point
 * between ghost and mirror.  Periodic axes wrap.  The x rule is applied
 * first, so corner ghosts use the y-wall rule at the mirrored column. */
static double ghost_value(const orc_state* s, const double* X, int kind, int i, int j)
{
    const orc_case* c = &s->c;
    const int nx = s->nx, ny = s->ny;
    if (!c->wall[0]) i = ((i % nx) + nx) % nx;
    if (!c->wall[2]) j = ((j % ny) + ny) % ny;
    if (i < 0 || i >= nx) {
        const int side = (i < 0) ? 0 : 1;
        const int im = (i < 0) ? -1 - i : 2 * nx - 1 - i;
        double v = ghost_value(s, X, kind, im, j);
        if (dirichlet_side(c, kind, side)) v = 2.0 * wall_value(c, kind, side, side ? nx - 0.5 : -0.5) - v;
        return v;
    }
    if (j < 0 || j >= ny) {
        const int side = (j < 0) ? 2 : 3;
        const int jm = (j < 0) ? -1 - j : 2 * ny - 1 - j;
        double v = X[(size_t)jm * nx + i];
        if (dirichlet_side(c, kind, side)) v = 2.0 * wall_value(c, kind, side, (double)i) - v;
        return v;
    }
    return X[(size_t)j * nx + i];
}

static void extend(const orc_state* s, const double* X, double* XE, int kind, int depth)
{
#pragma omp parallel for schedule(static)
    for (int j = -depth; j < s->ny + depth; ++j)
        for (int i = -depth; i < s->nx + depth; ++i) XE[eidx(s, i, j)] = ghost_value(s, X, kind, i, j);
}

/* Isotropic finite difference (the stencil the paper takes from Kumar 2004):
 *   d_a X(x) = (1/cs2) sum_alpha w_alpha e_alpha,a X(x + e_alpha),
 * evaluated in the equivalent difference form
 *   (1/cs2) sum_alpha w_alpha e_alpha,a [X(x + e_alpha) - X(x)]
 * (sum_alpha w_alpha e_alpha = 0), which keeps its accuracy where the gradient
 * is small against X itself (bubble centres, bulk): the differences of nearby
 * values are exact, the weighted sum of O(X) terms is not. */
static void iso_grad_ext(const orc_state* s, const double* XE, int i, int j, double* gx, double* gy)
{
    const double X0 = XE[eidx(s, i, j)];
    double ax = 0.0, ay = 0.0;
    for (int a = 1; a < 9; ++a) {
        const double d = XE[eidx(s, i + EX[a], j + EY[a])] - X0;
        ax += WT[a] * EX[a] * d;
        ay += WT[a] * EY[a] * d;
    }
    *gx = ax / CS2;
    *gy = ay / CS2;
}

void orc_grad_periodic(const double* X, int32_t nx, int32_t ny, double* gx, double* gy)
{
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double ax = 0.0, ay = 0.0;
            const double X0 = X[(size_t)j * nx + i];
            for (int a = 1; a < 9; ++a) {
                const int ii = ((i + EX[a]) % nx + nx) % nx, jj = ((j + EY[a]) % ny + ny) % ny;
                const double v = X[(size_t)jj * nx + ii] - X0;
                ax += WT[a] * EX[a] * v;
                ay += WT[a] * EY[a] * v;
            }
            gx[(size_t)j * nx + i] = ax / CS2;
            gy[(size_t)j * nx + i] = ay / CS2;
        }
}

/* ------------------------------------------------- surface tension law */
/* Sec. 2.1.  Law 1 is the printed equation of state,
 *   sigma = s0 + s0 beta (T/Tref) ln(1 - psi) + sT (T - Tref) + sTT (T - Tref)^2,
 * law 0 the multiplicative variant (quadratic-in-T clean tension times the
 * Langmuir factor 1 + beta ln(1 - psi/psi_inf)).  The logarithm's argument is
 * kept >= 1e-6 so that psi reaching psi_inf cannot produce a NaN. */
static double sigma_of(const orc_case* c, double T, double psi)
{
    const double dT = T - c->T_ref;
    double frac = psi / c->psi_inf;
    if (frac > 1.0 - 1e-6) frac = 1.0 - 1e-6;
    const double L = log(1.0 - frac);
    if (c->sigma_law == 1) return c->sigma0 + c->sigma0 * c->beta_s * (T / c->T_ref) * L + c->sigma_T * dT + c->sigma_TT * dT * dT;
    return (c->sigma0 + c->sigma_T * dT + c->sigma_TT * dT * dT) * (1.0 + c->beta_s * L);
}

/* dV/dphi / lambda for the regularised surfactant potential (Sec. 2):
 *   V/lambda = -(s/lambda)(8/W^2) phi^2 (1-phi)^2 + (w/lambda)/2 (phi - 1/2)^2
 * (phi_A = 0, phi_B = 1, so phi_o^2 - (phi - phi_m)^2 = phi (1 - phi)). */
static double dV_over_lambda(const orc_case* c, double phi)
{
    const double a = 8.0 / (c->W * c->W);
    return -c->s_lam * a * 2.0 * phi * (1.0 - phi) * (1.0 - 2.0 * phi) + c->w_lam * (phi - 0.5);
}

/* ---------------------------------------------------- macroscopic stage */
static void macro_stage(orc_state* s)
{
    const orc_case* c = &s->c;
    const int nx = s->nx, ny = s->ny;
    const size_t n = s->n;

    /* zeroth moments and the first moment of g (App. B-E) */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t k = (size_t)j * nx + i;
            double sf = 0, sg = 0, sh = 0, sq = 0, jx = 0, jy = 0;
            for (int a = 0; a < 9; ++a) {
                sf += s->pop[(0 * 9 + a) * n + k];
                const double g = s->pop[(1 * 9 + a) * n + k];
                sg += g;
                jx += g * EX[a];
                jy += g * EY[a];
                sh += s->pop[(2 * 9 + a) * n + k];
                sq += s->pop[(3 * 9 + a) * n + k];
            }
            s->phi[k] = sf;
            s->ps[k] = sg;
            s->jx[k] = jx;
            s->jy[k] = jy;
            s->T[k] = sh;
            s->psi[k] = sq;
        }

    extend(s, s->phi, s->phiE, GK_MIRROR, 2);
    extend(s, s->T, s->TE, GK_TEMP, 1);
    extend(s, s->psi, s->psiE, GK_PSI, 1);
    extend(s, s->ps, s->psE, GK_MIRROR, 1);

    /* grad phi, unit normal n = grad phi / |grad phi| and sigma on the domain
     * and its first ring (Sec. 3) */
#pragma omp parallel for schedule(static)
    for (int j = -1; j < ny + 1; ++j)
        for (int i = -1; i < nx + 1; ++i) {
            const size_t e = eidx(s, i, j);
            double gx, gy;
            iso_grad_ext(s, s->phiE, i, j, &gx, &gy);
            s->gxE[e] = gx;
            s->gyE[e] = gy;
            double mag = sqrt(gx * gx + gy * gy);
            if (mag < 1e-12) mag = 1e-12;
            s->nxE[e] = gx / mag;
            s->nyE[e] = gy / mag;
            s->sigE[e] = sigma_of(c, s->TE[e], s->psiE[e]);
        }

#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t k = (size_t)j * nx + i;
            const size_t e = eidx(s, i, j);
            const double phi = s->phi[k];
            const double gx = s->gxE[e], gy = s->gyE[e];
            const double g2 = gx * gx + gy * gy;
            const double nxv = s->nxE[e], nyv = s->nyE[e];

            /* curvature kappa = div n, isotropic divergence of the ring normals */
            double kap = 0.0;
            for (int a = 1; a < 9; ++a) {
                const size_t en = eidx(s, i + EX[a], j + EY[a]);
                kap += WT[a] * (EX[a] * (s->nxE[en] - nxv) + EY[a] * (s->nyE[en] - nyv));
            }
            kap /= CS2;

            /* CSF surface force (Sec. 3): delta_s = 1.5 W |grad phi|^2,
             * F_s = delta_s [ -sigma kappa n + grad sigma - n (n . grad sigma) ] */
            double dsx, dsy;
            iso_grad_ext(s, s->sigE, i, j, &dsx, &dsy);
            const double sig = s->sigE[e];
            const double ds = 1.5 * c->W * g2;
            const double ndots = nxv * dsx + nyv * dsy;
            const double Fsx = ds * (-sig * kap * nxv + dsx - nxv * ndots);
            const double Fsy = ds * (-sig * kap * nyv + dsy - nyv * ndots);

            /* density, viscosity: linear in phi between ambient (phi = 0) and
             * bubble (phi = 1) */
            const double rho = c->rho_A + phi * (c->rho_B - c->rho_A);
            const double mu = c->rho_A * c->nu_A + phi * (c->rho_B * c->nu_B - c->rho_A * c->nu_A);
            const double nu = mu / rho;
            const double alpha = c->alpha_A + phi * (c->alpha_B - c->alpha_A);

            /* pressure force F_p = -grad(p - rho cs2), p taken as the
             * zeroth moment of g before its force correction */
            double dpx, dpy;
            iso_grad_ext(s, s->psE, i, j, &dpx, &dpy);
            const double Fpx = -dpx + CS2 * (c->rho_B - c->rho_A) * gx;
            const double Fpy = -dpy + CS2 * (c->rho_B - c->rho_A) * gy;

            /* total force: surface + external (constant part and buoyancy) */
            const double Ftx = Fsx + c->Fext_x;
            const double Fty = Fsy + c->Fext_y - (rho - c->rho_A) * c->gravity;

            /* velocity and pressure (App. C) */
            const double ux = (s->jx[k] + 0.5 * CS2 * Ftx) / (rho * CS2);
            const double uy = (s->jy[k] + 0.5 * CS2 * Fty) / (rho * CS2);
            const double p = s->ps[k] + 0.5 * (Fpx * ux + Fpy * uy);

            /* adsorption/solubility driving R = grad V (chain rule) */
            const double dV = dV_over_lambda(c, phi);

            s->rho[k] = rho;
            s->ux[k] = ux;
            s->uy[k] = uy;
            s->p[k] = p;
            s->kap[k] = kap;
            s->Fsx[k] = Fsx;
            s->Fsy[k] = Fsy;
            s->Fpx[k] = Fpx;
            s->Fpy[k] = Fpy;
            s->Ftx[k] = Ftx;
            s->Fty[k] = Fty;
            s->Rx[k] = dV * gx;
            s->Ry[k] = dV * gy;
            s->omnu[k] = 1.0 / (nu / CS2 + 0.5);
            s->omT[k] = 1.0 / (alpha / CS2 + 0.5);
        }
}

/* ------------------------------------------------------------ collision */
static void collide_all(orc_state* s)
{
    const orc_case* c = &s->c;
    const int nx = s->nx, ny = s->ny;
    const size_t n = s->n;
    const double om_phi = 1.0 / (c->M_phi / CS2 + 0.5);
    const double om_psi = 1.0 / (c->D_psi / CS2 + 0.5);

#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t k = (size_t)j * nx + i;
            const size_t e = eidx(s, i, j);
            const double ux = s->ux[k], uy = s->uy[k];
            double in[9], out[9];

            /* f: phase field (App. B); first-order equilibrium is the
             * sharpening flux M_phi theta n, theta = 4 phi (1 - phi) / W. */
            const double phi = s->phi[k];
            const double theta = 4.0 * phi * (1.0 - phi) / c->W;
            for (int a = 0; a < 9; ++a) in[a] = s->pop[(0 * 9 + a) * n + k];
            orc_collide_ad(in, phi, c->M_phi * theta * s->nxE[e], c->M_phi * theta * s->nyE[e], om_phi, ux, uy, out);
            for (int a = 0; a < 9; ++a) s->post[(0 * 9 + a) * n + k] = out[a];

            /* g: two-fluid pressure/velocity (App. C) */
            for (int a = 0; a < 9; ++a) in[a] = s->pop[(1 * 9 + a) * n + k];
            orc_collide_g(in, s->p[k], s->rho[k], ux, uy, s->Ftx[k], s->Fty[k], s->Fpx[k], s->Fpy[k], s->omnu[k], out);
            for (int a = 0; a < 9; ++a) s->post[(1 * 9 + a) * n + k] = out[a];

            /* h: temperature (App. D) */
            for (int a = 0; a < 9; ++a) in[a] = s->pop[(2 * 9 + a) * n + k];
            orc_collide_ad(in, s->T[k], 0.0, 0.0, s->omT[k], ux, uy, out);
            for (int a = 0; a < 9; ++a) s->post[(2 * 9 + a) * n + k] = out[a];

            /* q: surfactant (App. E).  Reading: the first-order equilibrium is
             * -m_psi psi (1 - psi) R with m_psi = D_psi / lambda, so that the
             * recovered equation has diffusivity lambda m_psi = D_psi =
             * cs2 (1/omega_psi - 1/2) and adsorption flux m_psi psi (1-psi) R. */
            const double psi = s->psi[k];
            const double mflux = -c->D_psi * psi * (1.0 - psi);
            for (int a = 0; a < 9; ++a) in[a] = s->pop[(3 * 9 + a) * n + k];
            orc_collide_ad(in, psi, mflux * s->Rx[k], mflux * s->Ry[k], om_psi, ux, uy, out);
            for (int a = 0; a < 9; ++a) s->post[(3 * 9 + a) * n + k] = out[a];
        }
}

/* ------------------------------------------------------------ streaming */
/* X_a(x, t+1) = X~_a(x - e_a, t).  Where x - e_a lies beyond a wall:
 * halfway bounce-back X_a(x) = X~_abar(x) (no slip, zero flux), or for a
 * Dirichlet scalar the anti-bounce-back X_a(x) = -X~_abar(x) + 2 w_a X_w,
 * X_w taken at the link midpoint x - e_a/2.  When the source lies beyond both
 * a y-wall and an x-wall (corner links) the y-wall's rule applies. */
static void stream(orc_state* s)
{
    const orc_case* c = &s->c;
    const int nx = s->nx, ny = s->ny;
    const size_t n = s->n;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t k = (size_t)j * nx + i;
            for (int a = 0; a < 9; ++a) {
                int si = i - EX[a], sj = j - EY[a];
                if (!c->wall[0]) si = (si + nx) % nx;
                if (!c->wall[2]) sj = (sj + ny) % ny;
                const int outy = (sj < 0 || sj >= ny), outx = (si < 0 || si >= nx);
                if (!outx && !outy) {
                    const size_t ks = (size_t)sj * nx + si;
                    for (int set = 0; set < 4; ++set) s->pop[(set * 9 + a) * n + k] = s->post[(set * 9 + a) * n + ks];
                    continue;
                }
                const int side = outy ? (sj < 0 ? 2 : 3) : (si < 0 ? 0 : 1);
                const int b = OPP[a];
                s->pop[(0 * 9 + a) * n + k] = s->post[(0 * 9 + b) * n + k];
                s->pop[(1 * 9 + a) * n + k] = s->post[(1 * 9 + b) * n + k];
                if (c->t_bc[side] == 1) {
                    const double xm = (double)i - 0.5 * EX[a];
                    s->pop[(2 * 9 + a) * n + k] = -s->post[(2 * 9 + b) * n + k] + 2.0 * WT[a] * wall_T(c, xm);
                } else {
                    s->pop[(2 * 9 + a) * n + k] = s->post[(2 * 9 + b) * n + k];
                }
                if (c->psi_bc[side] == 1)
                    s->pop[(3 * 9 + a) * n + k] = -s->post[(3 * 9 + b) * n + k] + 2.0 * WT[a] * c->psi_w[side];
                else
                    s->pop[(3 * 9 + a) * n + k] = s->post[(3 * 9 + b) * n + k];
            }
        }
}

void orc_stream_only(orc_state* s, const double* post, double* out)
{
    memcpy(s->post, post, 36 * s->n * sizeof(double));
    stream(s);
    memcpy(out, s->pop, 36 * s->n * sizeof(double));
}

void orc_step(orc_state* s, int64_t nsteps)
{
    for (int64_t t = 0; t < nsteps; ++t) {
        macro_stage(s);
        collide_all(s);
        stream(s);
        s->step++;
    }
}

void orc_fields(orc_state* s, double* out)
{
    macro_stage(s);
    const size_t n = s->n;
    memcpy(out + 0 * n, s->phi, n * sizeof(double));
    memcpy(out + 1 * n, s->p, n * sizeof(double));
    memcpy(out + 2 * n, s->ux, n * sizeof(double));
    memcpy(out + 3 * n, s->uy, n * sizeof(double));
    memcpy(out + 4 * n, s->T, n * sizeof(double));
    memcpy(out + 5 * n, s->psi, n * sizeof(double));
}

void orc_intermediates(orc_state* s, double* out)
{
    macro_stage(s);
    const size_t n = s->n;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            const size_t k = (size_t)j * s->nx + i;
            const size_t e = eidx(s, i, j);
            out[0 * n + k] = s->gxE[e];
            out[1 * n + k] = s->gyE[e];
            out[2 * n + k] = s->kap[k];
            out[3 * n + k] = s->sigE[e];
            out[4 * n + k] = s->Fsx[k];
            out[5 * n + k] = s->Fsy[k];
            out[6 * n + k] = s->Fpx[k];
            out[7 * n + k] = s->Fpy[k];
            out[8 * n + k] = s->Rx[k];
            out[9 * n + k] = s->Ry[k];
            out[10 * n + k] = s->omnu[k];
            out[11 * n + k] = s->ps[k];
        }
}

/* Diagnostics: totals of phi and psi; bubble centroid and migration velocity
 * as phi-weighted means (the paper's "average velocity inside the bubble");
 * mean pressure where phi >= 0.99 (inside) and phi <= 0.01 (outside);
 * extrema; count of non-finite populations. */
void orc_diag(orc_state* s, double* out)
{
    macro_stage(s);
    const size_t n = s->n;
    double sphi = 0, spsi = 0, sx = 0, sy = 0, su = 0, sv = 0, pin = 0, pout = 0;
    double nin = 0, nout = 0;
    double phmin = INFINITY, phmax = -INFINITY, psmin = INFINITY, psmax = -INFINITY;
    double bad = 0;
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            const size_t k = (size_t)j * s->nx + i;
            const double ph = s->phi[k];
            sphi += ph;
            spsi += s->psi[k];
            sx += i * ph;
            sy += j * ph;
            su += s->ux[k] * ph;
            sv += s->uy[k] * ph;
            if (ph >= 0.99) {
                pin += s->p[k];
                nin += 1;
            }
            if (ph <= 0.01) {
                pout += s->p[k];
                nout += 1;
            }
            if (ph < phmin) phmin = ph;
            if (ph > phmax) phmax = ph;
            if (s->psi[k] < psmin) psmin = s->psi[k];
            if (s->psi[k] > psmax) psmax = s->psi[k];
        }
    for (size_t k = 0; k < 36 * n; ++k)
        if (!isfinite(s->pop[k])) bad += 1;
    out[0] = sphi;
    out[1] = spsi;
    out[2] = sx / sphi;
    out[3] = sy / sphi;
    out[4] = su / sphi;
    out[5] = sv / sphi;
    out[6] = nin > 0 ? pin / nin : 0.0;
    out[7] = nout > 0 ? pout / nout : 0.0;
    out[8] = phmin;
    out[9] = phmax;
    out[10] = psmin;
    out[11] = psmax;
    out[12] = bad;
    out[13] = (double)s->step;
}
