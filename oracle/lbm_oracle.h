/*
 * lbm_oracle.h -- plain FP64 CPU oracle of the coupled central-moment lattice
 * Boltzmann step of Elbousefi, Schupbach, Premnath & Welch, "Investigation of
 * surfactant-laden bubble migration dynamics in self-rewetting fluids using
 * lattice Boltzmann method" (arXiv 2408.00146).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.  Only
 * the test-suite, the package's smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant with
 * the GPU library and includes nothing from it.
 *
 * Units are lattice units throughout (dx = dt = 1).  All arrays are row-major
 * with x fastest: index = y*nx + x.  Populations are laid out
 * [set 0..3 = f, g, h, q][direction 0..8][y][x].
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem statement (Sec. 2, Sec. 2.1, Appendices B-E), lattice units. */
typedef struct orc_case {
    int32_t nx, ny;
    int32_t wall[4];     /* xmin, xmax, ymin, ymax: 1 = no-slip wall, 0 = periodic (pairs must agree) */
    int32_t t_bc[4];     /* per wall: 0 = zero flux, 1 = Dirichlet T_w(x) = T0 + gradT*(x - xT0) */
    int32_t psi_bc[4];   /* per wall: 0 = zero flux, 1 = Dirichlet psi_w[side] */
    double  psi_w[4];
    double  T0, gradT, xT0;
    int32_t sigma_law;   /* 0: (s0 + sT dT + sTT dT^2)(1 + beta ln(1 - psi/psi_inf)),  1: Eq. of Sec. 2.1 */
    int32_t init_kind;   /* 0 circular bubble, 1 slab |y - yc| < R, 2 uniform phi = 0 */
    double  sigma0, sigma_T, sigma_TT, T_ref, beta_s, psi_inf;
    double  rho_A, rho_B, nu_A, nu_B, alpha_A, alpha_B, D_psi, M_phi, W;
    double  s_lam, w_lam;  /* s/lambda and w/lambda of the surfactant chemical potential */
    double  Fext_x, Fext_y, gravity;
    double  xc, yc, R, psi_bulk, psi_band;
    double  psi_gradx;   /* initial psi adds psi_gradx (x - xT0): linear background along x */
    double  phi_noise;
    double  p_jump;      /* initial pressure p = p_jump (3 phi^2 - 2 phi^3) of the clean phi (0: p = 0) */
    uint64_t seed;
} orc_case;

/* Number of doubles written by orc_diag. */
#define ORC_NDIAG 14
/* diag layout: 0 sum phi, 1 sum psi, 2 xc, 3 yc, 4 ux_b, 5 uy_b, 6 p_in, 7 p_out,
 *              8 phi_min, 9 phi_max, 10 psi_min, 11 psi_max, 12 nonfinite count, 13 step */

typedef struct orc_state orc_state;

/* Returns NULL and writes a message to orc_error() when the case is invalid. */
orc_state* orc_create(const orc_case* c);
void       orc_free(orc_state* s);
const char* orc_error(void);

/* Reset populations to the rest equilibrium of given phi, T, psi (p = 0, u = 0). */
void orc_load_fields(orc_state* s, const double* phi, const double* T, const double* psi);
/* Advance n time steps. */
void orc_step(orc_state* s, int64_t n);
int64_t orc_steps_done(const orc_state* s);
/* Macroscopic fields of the current state: out[6][ny][nx] = phi, p, ux, uy, T, psi. */
void orc_fields(orc_state* s, double* out);
/* Intermediate coupling fields: out[12][ny][nx] =
 * dphi/dx, dphi/dy, kappa, sigma, Fs_x, Fs_y, Fp_x, Fp_y, R_x/lambda, R_y/lambda, omega_nu, p_star. */
void orc_intermediates(orc_state* s, double* out);
void orc_get_populations(const orc_state* s, double* out);
void orc_set_populations(orc_state* s, const double* in);
void orc_diag(orc_state* s, double* out);
int  orc_threads(void);

/* Pieces exposed for unit pins. */
void orc_matrix_P(double out[81]);
void orc_matrix_Pinv(double out[81]);
void orc_matrix_F(double ux, double uy, double out[81]);
void orc_matrix_Finv(double ux, double uy, double out[81]);
void orc_eq_g(double p, double rho, double ux, double uy, double out[9]);
void orc_source_g(double Ftx, double Fty, double Fpx, double Fpy, double ux, double uy, double out[9]);
void orc_collide_g(const double g[9], double p, double rho, double ux, double uy,
                   double Ftx, double Fty, double Fpx, double Fpy, double omega_nu, double out[9]);
/* Advection-diffusion collision shared by f, h, q: zeroth moment X, first-order central
 * equilibrium (jx, jy), first-order relaxation rate omega1, all higher rates 1. */
void orc_collide_ad(const double pop[9], double X, double jx, double jy, double omega1,
                    double ux, double uy, double out[9]);
/* Streaming alone: take `post` ([4][9][ny][nx]) as the post-collision
 * populations, stream them with the wall rules, and write the result to
 * `out`; the state's populations become that result. */
void orc_stream_only(orc_state* s, const double* post, double* out);
/* k-th output (k = 0, 1, ...) of the splitmix64 generator seeded with `seed`
 * (the noise source of the initial phase field). */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k);
/* Isotropic gradient of a periodic nx*ny field. */
void orc_grad_periodic(const double* X, int32_t nx, int32_t ny, double* gx, double* gy);

#ifdef __cplusplus
}
#endif
#endif
