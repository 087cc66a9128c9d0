// lbm_device.hpp -- gfx950 device code of the coupled central-moment LB step
// (arXiv 2408.00146): four D2Q9 sets f (phase field, App. B), g (two-fluid
// pressure/velocity, App. C), h (temperature, App. D), q (surfactant, App. E),
// coupled through the isotropic-gradient force terms of Sec. 2-3.
//
// One workgroup owns one BX x BY tile of one case.  Per time step it
//   1. pulls (streams) populations from the source buffer for the tile plus a
//      halo and reduces them to phi (2-node halo), p*, sigma(T, psi) (1-node
//      halo) in LDS;
//   2. forms the interface normal on the tile plus 1-node halo in LDS;
//   3. per own node: curvature, CSF force, pressure force, velocity,
//      pressure, the four central-moment collisions, store into the
//      destination buffer (pull ping-pong: every node writes only itself).
// Populations are SoA planes [set][dir][y][pitch] so that a wavefront of 64
// consecutive x reads/writes contiguous memory.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ------------------------------------------------------------- lattice
// D2Q9: e = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
__host__ __device__ constexpr int ex(int a) { return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0); }
__host__ __device__ constexpr int ey(int a) { return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0); }
__host__ __device__ constexpr int opp(int a) { return a == 0 ? 0 : (a <= 4 ? ((a + 1) % 4 + 1) : ((a - 5 + 2) % 4 + 5)); }
__host__ __device__ constexpr double wt(int a) { return a == 0 ? 4.0 / 9.0 : (a <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }

enum { SET_F = 0, SET_G = 1, SET_H = 2, SET_Q = 3 };
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP16S = 2 };

// ------------------------------------------------------- case parameters
// Device copy of one case, precomputed on the host.
struct CaseDev {
    int32_t nx, ny, pitch, prec;
    int32_t wallx, wally, law, refs;  // refs: populations stored as deviations from w*X_ref
    int32_t tbc[4], pbc[4];
    double psi_w[4];
    double T0, gradT, xT0;
    double s0, sT, sTT, Tref, beta, inv_psi_inf;
    double rhoA, drho, muA, dmu, alphaA, dalpha;
    double om_phi, om_psi, Mphi, W, Dpsi, s_lam, w_lam;
    double Fx, Fy, grav;
    double ref_q, scale, inv_scale;
    int64_t plane;      // elements per (set, dir) plane = ny * pitch
    int64_t max_steps;  // <= 0: unlimited
    void* buf[2];       // ping-pong population buffers
};

struct TileRec {
    int32_t c, x0, y0, pad;
};

// Per-case constants in the compute type, loaded once per tile.
template <typename R>
struct Ctx {
    int nx, ny, pitch, wallx, wally, law, refs;
    int tbc, pbc;  // bit s set: Dirichlet T / psi on side s (no dynamic array indexing: keeps Ctx in registers)
    int64_t plane;
    const double* psi_w;  // wall values read from global memory (a select over struct fields would defeat SROA)
    R T0, gradT, xT0;
    R s0, sT, sTT, Tref, beta, inv_psi_inf;
    R rhoA, drho, muA, dmu, alphaA, dalpha;
    R om_phi, om_psi, Mphi, W, Dpsi, s_lam, w_lam;
    R Fx, Fy, grav, ref_q, scale, inv_scale;

    __device__ void load(const CaseDev& c)
    {
        nx = c.nx; ny = c.ny; pitch = c.pitch; wallx = c.wallx; wally = c.wally; law = c.law; refs = c.refs;
        plane = c.plane;
        tbc = (c.tbc[0] ? 1 : 0) | (c.tbc[1] ? 2 : 0) | (c.tbc[2] ? 4 : 0) | (c.tbc[3] ? 8 : 0);
        pbc = (c.pbc[0] ? 1 : 0) | (c.pbc[1] ? 2 : 0) | (c.pbc[2] ? 4 : 0) | (c.pbc[3] ? 8 : 0);
        psi_w = c.psi_w;
        T0 = R(c.T0); gradT = R(c.gradT); xT0 = R(c.xT0);
        s0 = R(c.s0); sT = R(c.sT); sTT = R(c.sTT); Tref = R(c.Tref); beta = R(c.beta); inv_psi_inf = R(c.inv_psi_inf);
        rhoA = R(c.rhoA); drho = R(c.drho); muA = R(c.muA); dmu = R(c.dmu); alphaA = R(c.alphaA); dalpha = R(c.dalpha);
        om_phi = R(c.om_phi); om_psi = R(c.om_psi); Mphi = R(c.Mphi); W = R(c.W); Dpsi = R(c.Dpsi);
        s_lam = R(c.s_lam); w_lam = R(c.w_lam); Fx = R(c.Fx); Fy = R(c.Fy); grav = R(c.grav);
        ref_q = R(c.ref_q); scale = R(c.scale); inv_scale = R(c.inv_scale);
    }
    __device__ bool t_dir(int side) const { return (tbc >> side) & 1; }
    __device__ bool p_dir(int side) const { return (pbc >> side) & 1; }
    __device__ R psi_wall(int side) const { return R(psi_w[side]); }
    // Imposed linear wall-temperature law (also the storage reference of h).
    __device__ R Tlaw(R x) const { return T0 + gradT * (x - xT0); }
    // Storage reference of h at node column x (0 when populations are raw).
    __device__ R Tref_x(int x) const { return refs ? Tlaw(R(x)) : R(0); }
    __device__ R qref() const { return refs ? ref_q : R(0); }
};

// ------------------------------------------------------------ storage codec
template <typename S, typename R>
__device__ __forceinline__ R dec(S v, R inv_scale);
template <>
__device__ __forceinline__ double dec<double, double>(double v, double) { return v; }
template <>
__device__ __forceinline__ float dec<float, float>(float v, float) { return v; }
template <>
__device__ __forceinline__ float dec<__half, float>(__half v, float inv_scale) { return __half2float(v) * inv_scale; }

template <typename S, typename R>
__device__ __forceinline__ S enc(R v, R scale);
template <>
__device__ __forceinline__ double enc<double, double>(double v, double) { return v; }
template <>
__device__ __forceinline__ float enc<float, float>(float v, float) { return v; }
template <>
__device__ __forceinline__ __half enc<__half, float>(float v, float scale) { return __float2half_rn(v * scale); }

// ----------------------------------------------------------- streaming
// Post-streaming population X_a at node (x, y), as a deviation from the
// storage reference of node (x, y): X_a(x) = X~_a(x - e_a) (pull).  A source
// beyond a wall gives halfway bounce-back X_a(x) = X~_abar(x), or for a
// Dirichlet scalar (h: T_w(x - e_a/2); q: psi_w) the anti-bounce-back
// X_a(x) = -X~_abar(x) + 2 w_a X_w.  A source beyond both a y-wall and an
// x-wall follows the y-wall's rule.
template <int SET, int A, typename S, typename R>
__device__ __forceinline__ R pull(const Ctx<R>& c, const S* __restrict__ src, int x, int y)
{
    constexpr int EX = ex(A), EY = ey(A);
    int sx = x - EX, sy = y - EY;
    if (EX != 0 && !c.wallx) sx = sx < 0 ? sx + c.nx : (sx >= c.nx ? sx - c.nx : sx);
    if (EY != 0 && !c.wally) sy = sy < 0 ? sy + c.ny : (sy >= c.ny ? sy - c.ny : sy);
    const bool outy = (EY != 0) && (sy < 0 || sy >= c.ny);
    const bool outx = (EX != 0) && (sx < 0 || sx >= c.nx);
    if (!outx && !outy) {
        const R v = dec<S, R>(src[(int64_t)(SET * 9 + A) * c.plane + (int64_t)sy * c.pitch + sx], c.inv_scale);
        if (SET == SET_H && EX != 0) {
            // re-reference from column sx to column x (h deviations only)
            if (c.refs) return v + R(wt(A)) * c.gradT * R(sx - x);
        }
        return v;
    }
    constexpr int B = opp(A);
    const R v = dec<S, R>(src[(int64_t)(SET * 9 + B) * c.plane + (int64_t)y * c.pitch + x], c.inv_scale);
    if (SET != SET_H && SET != SET_Q) return v;
    const int side = outy ? (sy < 0 ? 2 : 3) : (sx < 0 ? 0 : 1);
    if (SET == SET_H) {
        if (!c.t_dir(side)) return v;
        // 2 w_a (T_w(x - e_a/2) - Tref(x)); with the linear-law reference the
        // difference is exactly -gradT * ex / 2.
        const R d = c.refs ? R(-0.5) * c.gradT * R(EX) : c.Tlaw(R(x) - R(0.5) * R(EX));
        return -v + R(2.0 * wt(A)) * d;
    }
    if (!c.p_dir(side)) return v;
    return -v + R(2.0 * wt(A)) * (c.psi_wall(side) - c.qref());
}

template <int SET, typename S, typename R>
__device__ __forceinline__ void pull9(const Ctx<R>& c, const S* __restrict__ src, int x, int y, R v[9])
{
    v[0] = pull<SET, 0, S, R>(c, src, x, y);
    v[1] = pull<SET, 1, S, R>(c, src, x, y);
    v[2] = pull<SET, 2, S, R>(c, src, x, y);
    v[3] = pull<SET, 3, S, R>(c, src, x, y);
    v[4] = pull<SET, 4, S, R>(c, src, x, y);
    v[5] = pull<SET, 5, S, R>(c, src, x, y);
    v[6] = pull<SET, 6, S, R>(c, src, x, y);
    v[7] = pull<SET, 7, S, R>(c, src, x, y);
    v[8] = pull<SET, 8, S, R>(c, src, x, y);
}

template <typename R>
__device__ __forceinline__ R sum9(const R v[9])
{
    R s = R(0);
#pragma unroll
    for (int a = 0; a < 9; ++a) s += v[a];
    return s;
}

// --------------------------------------------------------- ghost nodes
// A node outside the lattice takes the value of its mirror node across the
// wall (zero normal gradient), or 2 X_w - X(mirror) on a Dirichlet wall;
// periodic axes wrap.  The y rule is applied at the mirrored column, then
// the x rule.
struct GhostMap {
    int ix, iy, xside, yside;
};

template <typename R>
__device__ __forceinline__ GhostMap ghost_map(const Ctx<R>& c, int gx, int gy)
{
    GhostMap m;
    gx = gx < -2 ? -2 : (gx > c.nx + 1 ? c.nx + 1 : gx);
    gy = gy < -2 ? -2 : (gy > c.ny + 1 ? c.ny + 1 : gy);
    if (!c.wallx) gx = gx < 0 ? gx + c.nx : (gx >= c.nx ? gx - c.nx : gx);
    if (!c.wally) gy = gy < 0 ? gy + c.ny : (gy >= c.ny ? gy - c.ny : gy);
    m.xside = -1;
    m.yside = -1;
    if (gx < 0) { m.xside = 0; gx = -1 - gx; }
    else if (gx >= c.nx) { m.xside = 1; gx = 2 * c.nx - 1 - gx; }
    if (gy < 0) { m.yside = 2; gy = -1 - gy; }
    else if (gy >= c.ny) { m.yside = 3; gy = 2 * c.ny - 1 - gy; }
    m.ix = gx;
    m.iy = gy;
    return m;
}

template <typename R>
__device__ __forceinline__ R ghost_T(const Ctx<R>& c, const GhostMap& m, R T)
{
    if (m.yside >= 0 && c.t_dir(m.yside)) T = R(2) * c.Tlaw(R(m.ix)) - T;
    if (m.xside >= 0 && c.t_dir(m.xside)) T = R(2) * c.Tlaw(m.xside ? R(c.nx) - R(0.5) : R(-0.5)) - T;
    return T;
}

template <typename R>
__device__ __forceinline__ R ghost_psi(const Ctx<R>& c, const GhostMap& m, R p)
{
    if (m.yside >= 0 && c.p_dir(m.yside)) p = R(2) * c.psi_wall(m.yside) - p;
    if (m.xside >= 0 && c.p_dir(m.xside)) p = R(2) * c.psi_wall(m.xside) - p;
    return p;
}

// ------------------------------------------------------ material laws
// Surface tension (Sec. 2.1): law 1 as printed, law 0 the multiplicative
// Langmuir variant; the log argument is floored at 1e-6.
template <typename R>
__device__ __forceinline__ R sigma_of(const Ctx<R>& c, R T, R psi)
{
    const R dT = T - c.Tref;
    R frac = psi * c.inv_psi_inf;
    frac = frac > R(1.0 - 1e-6) ? R(1.0 - 1e-6) : frac;
    const R L = log(R(1) - frac);
    if (c.law == 1) return c.s0 + c.s0 * c.beta * (T / c.Tref) * L + c.sT * dT + c.sTT * dT * dT;
    return (c.s0 + c.sT * dT + c.sTT * dT * dT) * (R(1) + c.beta * L);
}

// ----------------------------------------------------------- collisions
// Inverse raw-moment map P^-1 (App. F) from raw moments
// m = (00, 10, 01, 20, 02, 11, 21, 12, 22).
template <typename R>
__device__ __forceinline__ void raw_to_pop(const R m[9], R o[9])
{
    const R h = R(0.5), q = R(0.25);
    o[0] = m[0] - m[3] - m[4] + m[8];
    o[1] = h * (m[1] + m[3] - m[7] - m[8]);
    o[2] = h * (m[2] + m[4] - m[6] - m[8]);
    o[3] = h * (-m[1] + m[3] + m[7] - m[8]);
    o[4] = h * (-m[2] + m[4] + m[6] - m[8]);
    o[5] = q * (m[5] + m[6] + m[7] + m[8]);
    o[6] = q * (-m[5] + m[6] - m[7] + m[8]);
    o[7] = q * (m[5] - m[6] - m[7] + m[8]);
    o[8] = q * (-m[5] - m[6] + m[7] + m[8]);
}

// Advection-diffusion central-moment collision (f: App. B, h: App. D,
// q: App. E).  Post-collision central moments are
// (X, a_x, a_y, X/3, X/3, 0, 0, 0, X/9) with a = k1 + w1 (j_eq - k1), k1 the
// pre-collision first central moment.  Populations enter and leave as
// deviations d_a = X_a - w_a Xr from a reference Xr; with X = Xr + sum d:
//   d~ = w Xdev + P^-1 [ X dM(u) + A(u, a) ],
// dM(u) = F^-1(u)(1,0,0,1/3,1/3,0,0,0,1/9) minus its u = 0 value and
// A(u, a) = F^-1(u)(0, a_x, a_y, 0, ...).  With Xr = 0 this is the plain
// P^-1 F^-1(u) of the post-collision central moments.
template <typename R>
__device__ __forceinline__ void collide_ad(R d[9], R Xr, R jx, R jy, R w1, R ux, R uy)
{
    const R Xd = sum9(d);
    const R X = Xr + Xd;
    const R mx = d[1] - d[3] + d[5] - d[6] - d[7] + d[8];
    const R my = d[2] - d[4] + d[5] + d[6] - d[7] - d[8];
    const R kx = mx - ux * X, ky = my - uy * X;
    const R ax = kx + w1 * (jx - kx), ay = ky + w1 * (jy - ky);
    const R third = R(1.0 / 3.0);
    const R uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
    R v[9];
    v[0] = R(0);
    v[1] = X * ux + ax;
    v[2] = X * uy + ay;
    v[3] = X * uxx + R(2) * ux * ax;
    v[4] = X * uyy + R(2) * uy * ay;
    v[5] = X * uxy + uy * ax + ux * ay;
    v[6] = X * (uxx * uy + third * uy) + R(2) * uxy * ax + uxx * ay;
    v[7] = X * (ux * uyy + third * ux) + uyy * ax + R(2) * uxy * ay;
    v[8] = X * (uxx * uyy + third * (uxx + uyy)) + R(2) * uxy * uy * ax + R(2) * uxy * ux * ay;
    R o[9];
    raw_to_pop(v, o);
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = R(wt(a)) * Xd + o[a];
}

// Two-fluid central-moment collision (App. C): every moment relaxes with
// rate 1 except the deviatoric second moments (2d, 11) at omega_nu, and each
// takes (1 - w/2) times its source moment.
template <typename R>
__device__ __forceinline__ void collide_g(R g[9], R pstar, R jx, R jy, R p, R rho, R ux, R uy, R Ftx, R Fty,
                                          R Fpx, R Fpy, R om)
{
    const R cs2 = R(1.0 / 3.0);
    const R uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
    // pre-collision raw second moments -> central 2nd moments
    const R r20 = g[1] + g[3] + g[5] + g[6] + g[7] + g[8];
    const R r02 = g[2] + g[4] + g[5] + g[6] + g[7] + g[8];
    const R r11 = g[5] - g[6] + g[7] - g[8];
    const R e20 = r20 - R(2) * ux * jx + uxx * pstar;
    const R e02 = r02 - R(2) * uy * jy + uyy * pstar;
    const R e11 = r11 - uy * jx - ux * jy + uxy * pstar;
    // equilibria, varphi = p - rho cs2; the 22 moment is written as
    // p cs2^2 + varphi (cs2 (ux^2 + uy^2) + ux^2 uy^2) (same value, no cancellation)
    const R vp = p - rho * cs2;
    const R q00 = p, q10 = -vp * ux, q01 = -vp * uy;
    const R q20 = p * cs2 + vp * uxx, q02 = p * cs2 + vp * uyy, q11 = vp * uxy;
    const R q21 = -vp * (uxx + cs2) * uy, q12 = -vp * (uyy + cs2) * ux;
    const R q22 = p * cs2 * cs2 + vp * (cs2 * (uxx + uyy) + uxx * uyy);
    // source moments, Gamma00 = Fp . u
    const R G = Fpx * ux + Fpy * uy;
    const R s10 = cs2 * Ftx - ux * G, s01 = cs2 * Fty - uy * G;
    const R s20 = R(2) * cs2 * Fpx * ux + (uxx + cs2) * G;
    const R s02 = R(2) * cs2 * Fpy * uy + (uyy + cs2) * G;
    const R s11 = cs2 * (Fpx * uy + Fpy * ux) + uxy * G;
    // relaxation in the (00, 10, 01, 2s, 2d, 11, 21, 12, 22) basis
    const R h = R(0.5);
    const R t00 = q00 + h * G;
    const R t10 = q10 + h * s10;
    const R t01 = q01 + h * s01;
    const R t2s = (q20 + q02) + h * (s20 + s02);
    const R e2d = e20 - e02;
    const R t2d = e2d + om * ((q20 - q02) - e2d) + (R(1) - h * om) * (s20 - s02);
    const R t11 = e11 + om * (q11 - e11) + (R(1) - h * om) * s11;
    const R t20 = h * (t2s + t2d), t02 = h * (t2s - t2d);
    // back to raw moments: F^-1(u)
    R m[9];
    m[0] = t00;
    m[1] = ux * t00 + t10;
    m[2] = uy * t00 + t01;
    m[3] = uxx * t00 + R(2) * ux * t10 + t20;
    m[4] = uyy * t00 + R(2) * uy * t01 + t02;
    m[5] = uxy * t00 + uy * t10 + ux * t01 + t11;
    m[6] = uxx * uy * t00 + R(2) * uxy * t10 + uxx * t01 + uy * t20 + R(2) * ux * t11 + q21;
    m[7] = ux * uyy * t00 + uyy * t10 + R(2) * uxy * t01 + ux * t02 + R(2) * uy * t11 + q12;
    m[8] = uxx * uyy * t00 + R(2) * ux * uyy * t10 + R(2) * uxx * uy * t01 + uyy * t20 + uxx * t02 +
           R(4) * uxy * t11 + R(2) * uy * q21 + R(2) * ux * q12 + q22;
    raw_to_pop(m, g);
}

// Derivative of the surfactant potential over lambda (Sec. 2):
// V/lambda = -(s/lambda)(8/W^2) phi^2 (1-phi)^2 + (w/lambda)/2 (phi - 1/2)^2.
template <typename R>
__device__ __forceinline__ R dV_lam(const Ctx<R>& c, R phi)
{
    const R a = R(8) / (c.W * c.W);
    return -c.s_lam * a * R(2) * phi * (R(1) - phi) * (R(1) - R(2) * phi) + c.w_lam * (phi - R(0.5));
}

// ------------------------------------------------------------ tile body
enum { MODE_STEP = 0, MODE_MACRO = 1 };

// Output of the macro (diagnostic / export) mode.
struct MacroOut {
    double* fields;     // dense nx*ny planes, in mask-bit order; may be null
    uint32_t mask;
    double* partials;   // per-block diagnostic partial sums; may be null
};
enum { NDIAG_PART = 16 };

template <typename R, int BX, int BY>
struct Smem {
    static constexpr int W2 = BX + 4, H2 = BY + 4, W1 = BX + 2, H1 = BY + 2;
    R phi[H2 * W2];
    R ps[H1 * W1];
    R sig[H1 * W1];
    R nx[H1 * W1];
    R ny[H1 * W1];
};

template <typename R, typename S, int BX, int BY, int MODE>
__device__ __forceinline__ void tile_body(const Ctx<R>& c, int x0, int y0, const S* __restrict__ src, S* __restrict__ dst,
                          Smem<R, BX, BY>& sh, const MacroOut& mo, double* dacc)
{
    constexpr int NT = 256;
    constexpr int W2 = BX + 4, H2 = BY + 4, W1 = BX + 2;
    const int tid = threadIdx.x;
    const R cs2 = R(1.0 / 3.0), inv_cs2 = R(3);

    // ---- phase 1: phi on tile + 2 halo; p*, sigma on tile + 1 halo
    for (int k = tid; k < W2 * H2; k += NT) {
        const int lx = k % W2, ly = k / W2;
        const GhostMap m = ghost_map(c, x0 - 2 + lx, y0 - 2 + ly);
        R v[9];
        pull9<SET_F>(c, src, m.ix, m.iy, v);
        sh.phi[k] = sum9(v);
        if (lx >= 1 && lx <= BX + 2 && ly >= 1 && ly <= BY + 2) {
            const int e = (ly - 1) * W1 + (lx - 1);
            pull9<SET_G>(c, src, m.ix, m.iy, v);
            sh.ps[e] = sum9(v);  // zero normal gradient at walls: mirror value as is
            pull9<SET_H>(c, src, m.ix, m.iy, v);
            const R T = ghost_T(c, m, c.Tref_x(m.ix) + sum9(v));
            pull9<SET_Q>(c, src, m.ix, m.iy, v);
            const R psi = ghost_psi(c, m, c.qref() + sum9(v));
            sh.sig[e] = sigma_of(c, T, psi);
        }
    }
    __syncthreads();

    // ---- phase 2: unit normal n = grad phi / |grad phi| on tile + 1 halo
    for (int e = tid; e < W1 * (BY + 2); e += NT) {
        const int lx = e % W1 + 1, ly = e / W1 + 1;  // in phi (E2) coordinates
        const R* P = sh.phi;
        const R gx = (R(4) * (P[ly * W2 + lx + 1] - P[ly * W2 + lx - 1]) + P[(ly + 1) * W2 + lx + 1] -
                      P[(ly + 1) * W2 + lx - 1] + P[(ly - 1) * W2 + lx + 1] - P[(ly - 1) * W2 + lx - 1]) *
                     R(1.0 / 12.0);
        const R gy = (R(4) * (P[(ly + 1) * W2 + lx] - P[(ly - 1) * W2 + lx]) + P[(ly + 1) * W2 + lx + 1] -
                      P[(ly - 1) * W2 + lx + 1] + P[(ly + 1) * W2 + lx - 1] - P[(ly - 1) * W2 + lx - 1]) *
                     R(1.0 / 12.0);
        R mag = sqrt(gx * gx + gy * gy);
        mag = mag < R(1e-12) ? R(1e-12) : mag;
        sh.nx[e] = gx / mag;
        sh.ny[e] = gy / mag;
    }
    __syncthreads();

    // ---- phase 3: own nodes
    constexpr int ROWS = NT / BX;  // rows covered by the block per pass
    const int lx = tid % BX;
    for (int ly = tid / BX; ly < BY; ly += ROWS) {
        const int x = x0 + lx, y = y0 + ly;
        const bool live = (x < c.nx) && (y < c.ny);
        // stencil helpers (E2 coords: +2, E1 coords: +1)
        const int p2 = (ly + 2) * W2 + (lx + 2);
        const int p1 = (ly + 1) * W1 + (lx + 1);
        const R* P = sh.phi;
        const R phi = P[p2];
        const R gx = (R(4) * (P[p2 + 1] - P[p2 - 1]) + P[p2 + W2 + 1] - P[p2 + W2 - 1] + P[p2 - W2 + 1] -
                      P[p2 - W2 - 1]) * R(1.0 / 12.0);
        const R gy = (R(4) * (P[p2 + W2] - P[p2 - W2]) + P[p2 + W2 + 1] - P[p2 - W2 + 1] + P[p2 + W2 - 1] -
                      P[p2 - W2 - 1]) * R(1.0 / 12.0);
        const R nxv = sh.nx[p1], nyv = sh.ny[p1];
        // curvature: isotropic divergence of the normal field
        const R* NX = sh.nx;
        const R* NY = sh.ny;
        const R kap = (R(4) * (NX[p1 + 1] - NX[p1 - 1] + NY[p1 + W1] - NY[p1 - W1]) +
                       (NX[p1 + W1 + 1] - NX[p1 + W1 - 1] + NX[p1 - W1 + 1] - NX[p1 - W1 - 1]) +
                       (NY[p1 + W1 + 1] - NY[p1 - W1 + 1] + NY[p1 + W1 - 1] - NY[p1 - W1 - 1])) *
                      R(1.0 / 12.0);
        const R* SG = sh.sig;
        const R sig = SG[p1];
        const R dsx = (R(4) * (SG[p1 + 1] - SG[p1 - 1]) + SG[p1 + W1 + 1] - SG[p1 + W1 - 1] + SG[p1 - W1 + 1] -
                       SG[p1 - W1 - 1]) * R(1.0 / 12.0);
        const R dsy = (R(4) * (SG[p1 + W1] - SG[p1 - W1]) + SG[p1 + W1 + 1] - SG[p1 - W1 + 1] + SG[p1 + W1 - 1] -
                       SG[p1 - W1 - 1]) * R(1.0 / 12.0);
        const R* PS = sh.ps;
        const R pstar = PS[p1];
        const R dpx = (R(4) * (PS[p1 + 1] - PS[p1 - 1]) + PS[p1 + W1 + 1] - PS[p1 + W1 - 1] + PS[p1 - W1 + 1] -
                       PS[p1 - W1 - 1]) * R(1.0 / 12.0);
        const R dpy = (R(4) * (PS[p1 + W1] - PS[p1 - W1]) + PS[p1 + W1 + 1] - PS[p1 - W1 + 1] + PS[p1 + W1 - 1] -
                       PS[p1 - W1 - 1]) * R(1.0 / 12.0);

        // CSF surface force: 1.5 W |grad phi|^2 [ -sigma kappa n + (I - n n) grad sigma ]
        const R ds = R(1.5) * c.W * (gx * gx + gy * gy);
        const R nds = nxv * dsx + nyv * dsy;
        const R Fsx = ds * (-sig * kap * nxv + dsx - nxv * nds);
        const R Fsy = ds * (-sig * kap * nyv + dsy - nyv * nds);
        // properties linear in phi
        const R rho = c.rhoA + phi * c.drho;
        const R mu = c.muA + phi * c.dmu;
        const R omnu = R(1) / (mu / rho * inv_cs2 + R(0.5));
        const R alpha = c.alphaA + phi * c.dalpha;
        const R omT = R(1) / (alpha * inv_cs2 + R(0.5));
        // pressure force -grad(p* - rho cs2), total force
        const R Fpx = -dpx + cs2 * c.drho * gx;
        const R Fpy = -dpy + cs2 * c.drho * gy;
        const R Ftx = Fsx + c.Fx;
        const R Fty = Fsy + c.Fy - (rho - c.rhoA) * c.grav;

        if (!live) continue;

        // g: momentum, velocity and pressure
        R g[9];
        pull9<SET_G>(c, src, x, y, g);
        const R jx = g[1] - g[3] + g[5] - g[6] - g[7] + g[8];
        const R jy = g[2] - g[4] + g[5] + g[6] - g[7] - g[8];
        const R ux = (jx + R(0.5) * cs2 * Ftx) / (rho * cs2);
        const R uy = (jy + R(0.5) * cs2 * Fty) / (rho * cs2);
        const R p = pstar + R(0.5) * (Fpx * ux + Fpy * uy);
        const R dV = dV_lam(c, phi);

        if (MODE == MODE_MACRO) {
            R hv[9], qv[9], fv[9];
            pull9<SET_H>(c, src, x, y, hv);
            pull9<SET_Q>(c, src, x, y, qv);
            pull9<SET_F>(c, src, x, y, fv);
            const R T = c.Tref_x(x) + sum9(hv);
            const R psi = c.qref() + sum9(qv);
            if (mo.fields) {
                const int64_t n = (int64_t)c.nx * c.ny, k = (int64_t)y * c.nx + x;
                const R vals[18] = {phi, p, ux, uy, T, psi, gx, gy, kap, sig, Fsx, Fsy, Fpx, Fpy,
                                    dV * gx, dV * gy, omnu, pstar};
                int slot = 0;
#pragma unroll
                for (int b = 0; b < 18; ++b)
                    if (mo.mask & (1u << b)) mo.fields[(slot++) * n + k] = (double)vals[b];
            }
            if (dacc) {
                double bad = 0;
#pragma unroll
                for (int a = 0; a < 9; ++a)
                    bad += (isfinite((double)fv[a]) ? 0.0 : 1.0) + (isfinite((double)g[a]) ? 0.0 : 1.0) +
                           (isfinite((double)hv[a]) ? 0.0 : 1.0) + (isfinite((double)qv[a]) ? 0.0 : 1.0);
                const double dphi = (double)phi;
                dacc[0] += dphi;
                dacc[1] += (double)psi;
                dacc[2] += (double)x * dphi;
                dacc[3] += (double)y * dphi;
                dacc[4] += (double)ux * dphi;
                dacc[5] += (double)uy * dphi;
                if (dphi >= 0.99) { dacc[6] += (double)p; dacc[7] += 1.0; }
                if (dphi <= 0.01) { dacc[8] += (double)p; dacc[9] += 1.0; }
                dacc[10] += bad;
                dacc[11] = fmin(dacc[11], dphi);
                dacc[12] = fmax(dacc[12], dphi);
                dacc[13] = fmin(dacc[13], (double)psi);
                dacc[14] = fmax(dacc[14], (double)psi);
            }
            continue;
        }

        const int64_t o = (int64_t)y * c.pitch + x;
        collide_g(g, pstar, jx, jy, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, omnu);
#pragma unroll
        for (int a = 0; a < 9; ++a) dst[(int64_t)(SET_G * 9 + a) * c.plane + o] = enc<S, R>(g[a], c.scale);

        // f: phase field, first-order equilibrium M_phi theta n, theta = 4 phi (1 - phi) / W
        R f[9];
        pull9<SET_F>(c, src, x, y, f);
        const R mt = c.Mphi * R(4) * phi * (R(1) - phi) / c.W;
        collide_ad(f, R(0), mt * nxv, mt * nyv, c.om_phi, ux, uy);
#pragma unroll
        for (int a = 0; a < 9; ++a) dst[(int64_t)(SET_F * 9 + a) * c.plane + o] = enc<S, R>(f[a], c.scale);

        // h: temperature
        R hh[9];
        pull9<SET_H>(c, src, x, y, hh);
        collide_ad(hh, c.Tref_x(x), R(0), R(0), omT, ux, uy);
#pragma unroll
        for (int a = 0; a < 9; ++a) dst[(int64_t)(SET_H * 9 + a) * c.plane + o] = enc<S, R>(hh[a], c.scale);

        // q: surfactant, first-order equilibrium -D_psi psi (1 - psi) R/lambda
        R qq[9];
        pull9<SET_Q>(c, src, x, y, qq);
        const R psi = c.qref() + sum9(qq);
        const R mf = -c.Dpsi * psi * (R(1) - psi) * dV;
        collide_ad(qq, c.qref(), mf * gx, mf * gy, c.om_psi, ux, uy);
#pragma unroll
        for (int a = 0; a < 9; ++a) dst[(int64_t)(SET_Q * 9 + a) * c.plane + o] = enc<S, R>(qq[a], c.scale);
    }
}

}  // namespace lbm
