/*
 * lbm.h -- C ABI of the MI355X (gfx950) coupled central-moment lattice
 * Boltzmann step for surfactant-laden bubbles in self-rewetting fluids
 * (Elbousefi, Schupbach, Premnath & Welch, arXiv 2408.00146).
 *
 * One time step advances four D2Q9 distribution sets on a 2-D lattice:
 *   f  phase field phi, conservative Allen-Cahn equation   (App. B; Sec. 3)
 *   g  pressure p and velocity u of the two-fluid flow,     (App. C; Sec. 3)
 *      with capillary + Marangoni (CSF) force from sigma(T, psi)
 *   h  temperature T                                        (App. D)
 *   q  surfactant concentration psi                         (App. E; Sec. 2)
 * each by the central-moment collision of App. B-F, plus the isotropic
 * finite-difference gradients these need (Sec. 3), then streaming.
 *
 * Everything is in lattice units (dx = dt = 1).  All GPU work is enqueued on
 * the caller's HIP stream.  The caller owns the device workspace and the
 * stream; the library owns only the opaque host handle.  No function throws
 * across this boundary: each returns an lbm_status and, on failure, a
 * thread-local message is available from lbm_last_error().
 *
 * Field arrays exchanged through this ABI are FP64, row-major with x fastest
 * (index = y*nx + x), one nx*ny plane per field.  Populations are exchanged as
 * FP64 planes [set f,g,h,q][direction 0..8][y][x] in the D2Q9 order
 * e = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_E_INVAL = -1,     /* invalid argument or case parameter (message names it) */
    LBM_E_NOMEM = -2,     /* workspace too small / host allocation failed */
    LBM_E_DEVICE = -3,    /* a HIP call failed (message carries the HIP error) */
    LBM_E_NONFINITE = -4, /* lbm_reduce found NaN/Inf populations */
    LBM_E_STATE = -5      /* call not valid in the handle's current state */
} lbm_status;

/* Population storage per case.  The step computes in FP64 for LBM_FP64 and
 * in FP32 otherwise (FP64 only in the diagnostic reductions).  LBM_FP32 and
 * LBM_FP16S store deviations from the rest equilibrium of a per-node
 * reference, X_a - w_a X_ref(x), scaled by 1 (FP32) or 2^10 (FP16): X_ref is
 * the FP16-rounded phi, p*, T and psi of the node that wrote the value for f,
 * g, h and q (one 8-byte record of four FP16 values per node, next to each
 * population buffer).  LBM_FP64 stores the populations themselves.  Every
 * entry point exchanges full FP64 values. */
typedef enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16S = 2 } lbm_precision;

/* Surface tension equation of state (Sec. 2.1). */
typedef enum {
    LBM_SIGMA_MULT = 0,  /* (s0 + sT (T-Tref) + sTT (T-Tref)^2) * (1 + beta ln(1 - psi/psi_inf)) */
    LBM_SIGMA_PAPER = 1  /* s0 + s0 beta (T/Tref) ln(1 - psi) + sT (T-Tref) + sTT (T-Tref)^2     */
} lbm_sigma_law;

/* Initial interface. */
typedef enum {
    LBM_INIT_BUBBLE = 0, /* circle of radius R at (xc, yc), phi = 1 inside (bubble, fluid B) */
    LBM_INIT_SLAB = 1,   /* band |y - yc| < R, phi = 1 inside                                  */
    LBM_INIT_NONE = 2    /* phi = 0 everywhere (single ambient fluid)                          */
} lbm_init_kind;

/* One simulation case: the paper's problem statement (grid and walls Sec. 2;
 * wall temperature Sec. 2 and App. D; sigma law Sec. 2.1; property ratios and
 * groups Sec. 2.1, Sec. 6) in lattice units.  Sides are indexed
 * 0 = xmin, 1 = xmax, 2 = ymin, 3 = ymax. */
typedef struct lbm_case {
    int32_t nx, ny;          /* lattice nodes; each >= 4 */
    int32_t precision;       /* lbm_precision */
    int32_t sigma_law;       /* lbm_sigma_law */
    int32_t init_kind;       /* lbm_init_kind */
    uint8_t wall[4];         /* 1 = no-slip wall (halfway bounce-back), 0 = periodic; pairs must agree */
    uint8_t t_bc[4];         /* on walls: 0 = zero flux, 1 = Dirichlet T_w(x) = T0 + gradT (x - xT0) */
    uint8_t psi_bc[4];       /* on walls: 0 = zero flux, 1 = Dirichlet psi = psi_w[side] */
    uint8_t reserved0[4];
    double psi_w[4];
    double T0, gradT, xT0;   /* linear wall-temperature law; also the initial T field */
    double sigma0, sigma_T, sigma_TT, T_ref, beta_s, psi_inf;
    double rho_A, rho_B;     /* densities: ambient (phi = 0), bubble (phi = 1) */
    double nu_A, nu_B;       /* kinematic viscosities; mu(phi) is linear in phi */
    double alpha_A, alpha_B; /* thermal diffusivities, linear in phi */
    double D_psi;            /* surfactant diffusivity lambda m_psi */
    double M_phi;            /* phase-field mobility */
    double W;                /* interface width */
    double s_lam, w_lam;     /* s/lambda, w/lambda of the surfactant chemical potential */
    double Fext_x, Fext_y;   /* constant body force */
    double gravity;          /* buoyancy F_y -= (rho - rho_A) * gravity */
    double xc, yc, R;        /* initial interface geometry */
    double psi_bulk, psi_band; /* initial psi = psi_bulk + psi_gradx (x - xT0) + psi_band * 4 phi0 (1 - phi0) */
    double psi_gradx;        /* linear initial background of psi along x (between Dirichlet psi walls) */
    double phi_noise;        /* amplitude of uniform noise added to the initial phi */
    double p_jump;           /* initial pressure p = p_jump (3 phi0^2 - 2 phi0^3), phi0 without noise:
                                the pressure whose gradient carries the CSF force 1.5 W |grad phi|^2
                                of a tanh interface (Sec. 3), so a bubble may start at its Laplace
                                jump sigma/R; a density ratio of 1000 needs it (0 = uniform p = 0) */
    uint64_t seed;           /* noise: k-th splitmix64 output for node k = y*nx + x */
    int64_t max_steps;       /* step budget of this case within a batched run; <= 0 = unlimited */
} lbm_case;

/* Diagnostics (FP64), reduced on the GPU in a fixed order.  Sec. 6 follows a
 * bubble by its position and by the average velocity inside it; both are
 * taken phi-weighted here (x_c = sum x phi / sum phi, u_b = sum u phi /
 * sum phi), and the Laplace test of Sec. 5.1 compares the pressure inside
 * and outside the bubble (means over phi >= 0.99 and phi <= 0.01).
 * Sum phi and sum psi are the totals that the phase-field and surfactant
 * equations conserve (App. B, App. E). */
typedef struct lbm_diag {
    double mass_phi, mass_psi;   /* sum of phi, sum of psi over the lattice */
    double xc, yc;               /* phi-weighted centroid */
    double ux, uy;               /* phi-weighted mean velocity (bubble migration velocity) */
    double p_in, p_out;          /* mean p where phi >= 0.99, where phi <= 0.01 (0 if none) */
    double phi_min, phi_max, psi_min, psi_max;
    double nonfinite;            /* number of non-finite populations */
    int64_t step;                /* steps done by this case */
} lbm_diag;

/* Field selection for lbm_moments: fields are written in increasing bit order,
 * each as one FP64 nx*ny plane. */
enum {
    LBM_F_PHI = 1u << 0, LBM_F_P = 1u << 1, LBM_F_UX = 1u << 2, LBM_F_UY = 1u << 3,
    LBM_F_T = 1u << 4, LBM_F_PSI = 1u << 5,
    /* coupling fields of the step (Sec. 2-3, App. C) */
    LBM_F_DPHIX = 1u << 6, LBM_F_DPHIY = 1u << 7, LBM_F_KAPPA = 1u << 8, LBM_F_SIGMA = 1u << 9,
    LBM_F_FSX = 1u << 10, LBM_F_FSY = 1u << 11, LBM_F_FPX = 1u << 12, LBM_F_FPY = 1u << 13,
    LBM_F_RX = 1u << 14, LBM_F_RY = 1u << 15, LBM_F_OMEGA_NU = 1u << 16, LBM_F_PSTAR = 1u << 17,
    LBM_F_ALL_MACRO = (1u << 6) - 1,
    LBM_F_ALL = (1u << 18) - 1
};

typedef struct lbm_handle lbm_handle;

/* Bytes of device workspace needed for these cases (256-byte aligned start). */
size_t lbm_workspace_bytes(const lbm_case* cases, int32_t ncases);

/* Validate the cases, lay out the workspace, build the tile tables and set
 * the initial state of every case: the equilibrium tanh profile of the
 * phase field across the interface, phi = 1/2 + 1/2 tanh(2 d / W) with d
 * the signed distance to the circle or band (Sec. 3), plus seeded noise;
 * T on the linear wall law (Sec. 2); psi = psi_bulk + psi_gradx (x - xT0) +
 * psi_band 4 phi (1 - phi); p = p_jump (3 phi^2 - 2 phi^3); u = 0; every set
 * at its rest equilibrium (App. B-E at u = 0).  `workspace`
 * is device memory of at least lbm_workspace_bytes(), 256-byte aligned, owned
 * by the caller and used for everything the library keeps on the device (the
 * library allocates no device memory of its own; only the host-memory variants
 * of the field and population transfers below stage through a temporary
 * device buffer); `stream` is a hipStream_t (NULL =
 * default stream).  LBM_E_INVAL for: FP64 cases mixed with FP32/FP16S cases
 * in one handle; an LBM_FP16S case with nx < 64 (narrower than one tile row); a case whose population buffer (36 values per node in its
 * storage type, pitch nx rounded up to 64) exceeds 4 GiB, the reach of the
 * 32-bit buffer offsets; more than 2^28 nodes in a case.  On success *out
 * receives the handle. */
int lbm_init(const lbm_case* cases, int32_t ncases, void* workspace, size_t bytes, void* stream,
             lbm_handle** out);

/* Advance every case by nsteps time steps (each case stops at its
 * max_steps).  One step is the method's full update at every node: pull
 * streaming with the wall rules (Sec. 2), the moments phi, p*, T, psi, j,
 * the isotropic gradients and curvature (Sec. 3), sigma(T, psi) (Sec. 2.1),
 * the CSF and pressure forces, u and p (Sec. 3, App. C), and the four
 * central-moment collisions of App. B (f), C (g), D (h) and E (q) with the
 * transformation matrices of App. F.  Asynchronous on the handle's stream:
 * launches captured hipGraphs of up to 100 steps; returns LBM_E_DEVICE if a
 * launch fails (the handle then holds the state of the last completed step
 * on the device). */
int lbm_step(lbm_handle* h, int64_t nsteps);

/* Write the selected fields of one case at its current step into dst (FP64
 * planes, mask bit order).  dst_on_device != 0: dst is device memory, the
 * write is asynchronous on the stream.  dst_on_device == 0: dst is host
 * memory, the call stages through a temporary device buffer and synchronizes. */
int lbm_moments(lbm_handle* h, int32_t case_id, uint32_t field_mask, void* dst, int32_t dst_on_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * fields as lbm_moments with a host destination, staged through a fixed
 * device array of 64 MiB that the library holds on every device it runs on
 * until the process ends, instead of a temporary device buffer.  dst_host is
 * host memory of nf * nx * ny doubles (nf = set bits of field_mask, planes in
 * mask-bit order), owned by the caller.  No device memory is allocated or
 * freed.  LBM_E_INVAL when nf * nx * ny * 8 exceeds 64 MiB.  Synchronizes the
 * stream.  All calls on one GPU share its array and every call rewrites the
 * part it uses: calls that overlap in time on one device race. */
int lbm_moments_static(lbm_handle* h, int32_t case_id, uint32_t field_mask, void* dst_host);

/* Export / import the current populations of one case as FP64
 * [4][9][ny][nx] (checkpoint / restart).  Same dst/src conventions as
 * lbm_moments.  Import encodes into the case's storage precision. */
int lbm_get_populations(lbm_handle* h, int32_t case_id, void* dst, int32_t dst_on_device);
int lbm_set_populations(lbm_handle* h, int32_t case_id, const void* src, int32_t src_on_device);

/* Reset one case to the rest equilibrium of given FP64 fields phi, T, psi
 * (nx*ny each; p = 0, u = 0) and set its step count to 0. */
int lbm_load_fields(lbm_handle* h, int32_t case_id, const void* phi, const void* T, const void* psi,
                    int32_t src_on_device);

/* Reduce the diagnostics of one case (the quantities of struct lbm_diag,
 * Sec. 5.1 and Sec. 6) in FP64 on the GPU, in a fixed order, and copy them
 * to *out (host memory owned by the caller).  Synchronizes the stream.
 * Returns LBM_E_NONFINITE when any population is NaN/Inf; *out is filled
 * either way. */
int lbm_reduce(lbm_handle* h, int32_t case_id, lbm_diag* out);

/* Step-kernel configuration.  Index i < lbm_tile_count() selects one
 * workgroup per bx x by tile of the handle's tile table (kind 0), the tile
 * plus its halo staged in LDS each step:
 *   0: 64 x 8 tiles, 256 threads, two nodes per thread, each set pulled
 *      again right before its collision;
 *   1: 64 x 4 tiles, 256 threads, one node per thread, its 36 populations
 *      held in registers from the moment pass to the collision (the default
 *      of an FP64 handle);
 *   2: 64 x 8 tiles, 512 threads, one node per thread as in 1, with half
 *      the halo per node (the default of an FP32 / FP16-storage handle).
 * All compute the same step (results agree to rounding of identical
 * operations).  lbm_autotune times every configuration valid for this
 * handle's cases over trial_steps steps, in three interleaved rounds, and
 * keeps the one with the best time (a trial step re-reads the current state
 * and writes only the scratch half of the ping-pong pair, so the state is
 * unchanged); it synchronizes.  lbm_set_tile picks one by index;
 * lbm_tile_shape / lbm_tile_threads / lbm_tile_kind describe an index
 * (LBM_E_INVAL if out of range). */
int lbm_autotune(lbm_handle* h, int32_t trial_steps);
int lbm_tile_count(void);
int lbm_tile_shape(int32_t index, int32_t* bx, int32_t* by);
int lbm_tile_threads(int32_t index);
int lbm_tile_kind(int32_t index);
int lbm_set_tile(lbm_handle* h, int32_t index);
int lbm_get_tile(lbm_handle* h);

/* Launch mode of lbm_step: 1 = replay captured hipGraphs of step chunks
 * (default), 0 = plain kernel launches. */
int lbm_set_graph(lbm_handle* h, int32_t enable);

/* Steps done by one case. */
int64_t lbm_steps_done(lbm_handle* h, int32_t case_id);

/* Step timing with HIP events on the handle's stream.  lbm_set_kernel_timing
 * mode 1 launches every step on its own between two events (plain launches:
 * the duration of the step kernels alone); mode 2 records events around each
 * chunk as lbm_step launches it (captured graphs of up to 100 steps, i.e. the
 * production path, including the gaps between kernels and the step-counter
 * update); mode 0 turns timing off.  lbm_kernel_time_ms gives the average
 * per step over the last lbm_step call made while timing was on and the
 * number of steps it covered; LBM_E_STATE when no timed call exists,
 * LBM_E_INVAL for another mode. */
int lbm_set_kernel_timing(lbm_handle* h, int32_t enable);
int lbm_kernel_time_ms(lbm_handle* h, double* avg_ms, int64_t* launches);

/* Release the handle (not the caller's workspace).  Synchronizes the stream. */
int lbm_destroy(lbm_handle* h);

/* Message of the last failure on this thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
