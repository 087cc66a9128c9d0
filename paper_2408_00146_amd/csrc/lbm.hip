// lbm.hip -- gfx950 kernels and the C-ABI host runtime (include/lbm.h) of the
// coupled central-moment LB step of arXiv 2408.00146.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "lbm.h"
#include "lbm_device.hpp"

namespace lbm {

// Tile shapes compiled into the library (BX x BY nodes per 256-thread
// workgroup).  64 x 4: one node per thread, whose populations stay in
// registers from the moment pass to the collision; 64 x 8: two nodes per
// thread, each set pulled again right before its collision (the shape of the
// field-export kernel, kept as a step configuration for cross-checks).
struct Shape {
    int bx, by;
};
constexpr Shape kShapes[] = {{64, 8}, {64, 4}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
constexpr int kOwnShape = 1;
static_assert(kShapes[kOwnShape].bx * kShapes[kOwnShape].by == 256, "one node per thread");
constexpr int kMacroBX = 64, kMacroBY = 8;

// Step configurations: one workgroup of `nt` threads per tile of the table.
// With nt = bx * by each thread owns one node and holds its populations in
// registers from the moment pass to the collision; 64 x 8 tiles with 256
// threads pull each set again before its collision.  (A grid of resident
// workgroups walking the tile table, with or without issuing the next tile's
// loads ahead, was measured slower on MI355X and is not kept.)
struct Config {
    int shape, nt;
};
constexpr Config kConfigs[] = {{0, 256}, {1, 256}, {0, 512}};
constexpr int kNumConfigs = sizeof(kConfigs) / sizeof(kConfigs[0]);
// Configuration of a new handle: the 64 x 4 tile for FP64, the 64 x 8 tile of
// 512 threads otherwise (the fastest of each on the benchmark workloads).
constexpr int default_config(bool fp64) { return fp64 ? 1 : 2; }

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Each XCD works through one contiguous band of the tile table: the halo
// rows shared by vertically adjacent tiles then hit that XCD's own L2.
struct Band {
    int begin, end;   // tiles of this XCD's band
    int first, step;  // this workgroup's first tile and stride within it
};
__device__ __forceinline__ Band xcd_band(int b, int nblocks, int ntiles)
{
    const int xcd = b & 7, slot = b >> 3;
    const int q = ntiles >> 3, r = ntiles & 7;
    const int begin = xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q;
    const int len = q + (xcd < r ? 1 : 0);
    const int gq = nblocks >> 3, gr = nblocks & 7;
    return Band{begin, begin + len, begin + slot, gq + (xcd < gr ? 1 : 0)};
}

// A tile whose 3-node halo lies inside the lattice needs no wrap or wall logic.
__device__ __forceinline__ bool interior(const CaseDev& cd, int x0, int y0, int bx, int by)
{
    return x0 >= 3 && y0 >= 3 && x0 + bx + 3 <= cd.nx && y0 + by + 3 <= cd.ny;
}

template <typename R, typename S, int BX, int BY, int MODE, int NT = 256>
__device__ __forceinline__ void run_tile(const CaseDev& cd, const Ctx<R>& c, int x0, int y0, int b, Smem<R, BX, BY, sizeof(R) == 4>& sh,
                                         const MacroOut& mo, double* dacc)
{
    const View src{make_rsrc(cd.buf[b], cd.pop_bytes)};
    const View dst{make_rsrc(cd.buf[b ^ 1], MODE == MODE_STEP ? cd.pop_bytes : 0u)};
    const Rsrc rsrc = make_rsrc(cd.rbuf[b], cd.ref_bytes);
    const Rsrc rdst = make_rsrc(cd.rbuf[b ^ 1], MODE == MODE_STEP ? cd.ref_bytes : 0u);
    if (interior(cd, x0, y0, BX, BY))
        tile_body<R, S, BX, BY, MODE, true, NT>(c, x0, y0, src, dst, rsrc, rdst, sh, mo, dacc);
    else
        tile_body<R, S, BX, BY, MODE, false, NT>(c, x0, y0, src, dst, rsrc, rdst, sh, mo, dacc);
}

// Storage selection of a step launch: one storage type per kernel keeps the
// code of a single tile body in the instruction cache.  A handle that mixes
// FP32 and FP16 cases launches the FP16 and the FP32 kernels over the two
// parts of its tile table.
enum { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2 };

template <int ST>
using RealOf = typename std::conditional<ST == ST_F64, double, float>::type;
template <int ST>
using StoreOf = typename std::conditional<ST == ST_F64, double, typename std::conditional<ST == ST_F32, float, __half>::type>::type;

// Waves per SIMD asked of the compiler: four (<= 128 VGPRs) for the FP32 and
// FP16-storage tiles with one node per thread, three (<= 168) for the other
// FP32 tiles and the FP64 64 x 4 tile, two for the other FP64 tiles.
constexpr int waves_of(int st, int bx, int by, int nt)
{
    const bool own1 = bx * by == nt;
    return st == ST_F64 ? (own1 && nt == 256 ? 3 : 2) : (own1 ? 4 : 3);
}

// The step's budget check: a case stops at its max_steps.
__device__ __forceinline__ bool tile_live(const CaseDev* cases, const TileRec& tr, const int64_t* steps, int t, int& b)
{
    const CaseDev& cd = cases[tr.c];
    const int64_t s = steps[tr.c] + t;
    b = (int)(s & 1);
    return !(cd.max_steps > 0 && s >= cd.max_steps);
}

// One workgroup per tile of the table.
template <int ST, int BX, int BY, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(waves_of(ST, BX, BY, NT)))) void k_step(
    const CaseDev* __restrict__ cases, const TileRec* __restrict__ tiles, int ntiles, const int64_t* __restrict__ steps,
    int t)
{
    using R = RealOf<ST>;
    using S = StoreOf<ST>;
    __shared__ Smem<R, BX, BY, sizeof(R) == 4> sh;
    const Band bd = xcd_band(blockIdx.x, gridDim.x, ntiles);
    const TileRec tr = tiles[bd.first];
    int b;
    if (!tile_live(cases, tr, steps, t, b)) return;  // uniform over the block
    const CaseDev& cd = cases[tr.c];
    Ctx<R> c;
    c.template load<!(ST == ST_F32 && NT == 512)>(cd);
    const MacroOut mo{nullptr, 0u, nullptr};
    run_tile<R, S, BX, BY, MODE_STEP, NT>(cd, c, tr.x0, tr.y0, b, sh, mo, nullptr);
}

// Deterministic block reduction of the diagnostic partials: wave64 butterfly
// then a fixed-order pass over the 4 waves.  Slots 11, 13 are minima, 12, 14
// maxima, the rest sums.
__device__ __forceinline__ double combine(int k, double a, double b)
{
    if (k == 11 || k == 13) return fmin(a, b);
    if (k == 12 || k == 14) return fmax(a, b);
    return a + b;
}

__device__ void block_reduce(double v[NDIAG_PART], double (*red)[NDIAG_PART], double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NDIAG_PART; ++k) {
        double x = v[k];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) x = combine(k, x, __shfl_xor(x, m, 64));
        v[k] = x;
    }
    if (lane == 0)
        for (int k = 0; k < NDIAG_PART; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < NDIAG_PART) {
        const int k = threadIdx.x;
        double x = red[0][k];
        for (int w = 1; w < 4; ++w) x = combine(k, x, red[w][k]);
        out[k] = x;
    }
}

__device__ __forceinline__ void diag_init(double d[NDIAG_PART])
{
#pragma unroll
    for (int k = 0; k < NDIAG_PART; ++k) d[k] = 0.0;
    d[11] = INFINITY;
    d[12] = -INFINITY;
    d[13] = INFINITY;
    d[14] = -INFINITY;
}

template <typename R>
__global__ __launch_bounds__(256) void k_macro(const CaseDev* __restrict__ cases, const TileRec* __restrict__ tiles,
                                               int tile0, const int64_t* __restrict__ steps, int case_id,
                                               uint32_t mask, double* fields, double* partials)
{
    __shared__ Smem<R, kMacroBX, kMacroBY, sizeof(R) == 4> sh;
    __shared__ double red[4][NDIAG_PART];
    const TileRec tr = tiles[tile0 + blockIdx.x];
    const CaseDev& cd = cases[case_id];
    const int b = (int)(steps[case_id] & 1);
    Ctx<R> c;
    c.load(cd);
    const MacroOut mo{fields, mask, partials};
    double acc[NDIAG_PART];
    diag_init(acc);
    double* dacc = partials ? acc : nullptr;
    if constexpr (sizeof(R) == 8) {
        run_tile<double, double, kMacroBX, kMacroBY, MODE_MACRO>(cd, c, tr.x0, tr.y0, b, sh, mo, dacc);
    } else {
        if (cd.prec == PREC_FP16S)
            run_tile<float, __half, kMacroBX, kMacroBY, MODE_MACRO>(cd, c, tr.x0, tr.y0, b, sh, mo, dacc);
        else
            run_tile<float, float, kMacroBX, kMacroBY, MODE_MACRO>(cd, c, tr.x0, tr.y0, b, sh, mo, dacc);
    }
    if (partials) block_reduce(acc, red, partials + (int64_t)blockIdx.x * NDIAG_PART);
}

__global__ __launch_bounds__(256) void k_diag_final(const double* __restrict__ partials, int nblocks, double* out)
{
    __shared__ double red[4][NDIAG_PART];
    double acc[NDIAG_PART];
    diag_init(acc);
    for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
        for (int k = 0; k < NDIAG_PART; ++k) acc[k] = combine(k, acc[k], partials[(int64_t)b * NDIAG_PART + k]);
    block_reduce(acc, red, out);
}

__global__ void k_advance(const CaseDev* __restrict__ cases, int ncases, int64_t* steps, int64_t k)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncases) return;
    int64_t s = steps[i] + k;
    if (cases[i].max_steps > 0 && s > cases[i].max_steps) s = cases[i].max_steps;
    if (steps[i] < s) steps[i] = s;
}

// splitmix64 (Steele, Lea & Flood 2014), k-th output of the sequence seeded
// with `seed`; 53 high bits mapped to [-1, 1).
__device__ __forceinline__ double noise_unit(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

struct InitDev {
    int32_t kind, pad;
    double xc, yc, R, W, psi_bulk, psi_band, psi_gradx, xT0, phi_noise, p_jump;
    uint64_t seed;
};

// Clean initial phase profile: the tanh equilibrium of the conservative
// Allen-Cahn equation (Sec. 3) across the circle or band of radius R.
__device__ double init_phi(const InitDev& in, int x, int y)
{
    if (in.kind == 2) return 0.0;
    double d;
    if (in.kind == 1) d = in.R - fabs((double)y - in.yc);
    else d = in.R - sqrt(((double)x - in.xc) * ((double)x - in.xc) + ((double)y - in.yc) * ((double)y - in.yc));
    return 0.5 + 0.5 * tanh(2.0 * d / in.W);
}

// Where the post-streaming state of a case comes from: FP64 population
// planes [4][9][ny][nx], or FP64 fields phi/T/psi (rest equilibrium,
// g = 0 for p = 0, u = 0), or the built-in initial condition (tanh
// interface of Sec. 3 plus noise, linear wall law for T, psi background and band,
// p = p_jump (3 phi^2 - 2 phi^3) of the clean phi, the integral of the CSF
// weight 1.5 W |grad phi|^2 across a tanh interface; the rest equilibrium
// of g at u = 0 is w_a p).
struct StateSrc {
    const double* pops;
    const double *phi, *T, *psi;
    InitDev in;
};

__device__ double src_pop(const CaseDev& cd, const StateSrc& s, int set, int a, int x, int y)
{
    const int64_t n = (int64_t)cd.nx * cd.ny, k = (int64_t)y * cd.nx + x;
    if (s.pops) return s.pops[(int64_t)(set * 9 + a) * n + k];
    if (set == SET_G && (s.phi || s.in.p_jump == 0.0)) return 0.0;
    double X;
    if (s.phi) {
        X = set == SET_F ? s.phi[k] : (set == SET_H ? s.T[k] : s.psi[k]);
    } else if (set == SET_H) {
        X = cd.T0 + cd.gradT * ((double)x - cd.xT0);
    } else {
        const double pc = init_phi(s.in, x, y);
        if (set == SET_F) X = pc + s.in.phi_noise * noise_unit(s.in.seed, (uint64_t)k);
        else if (set == SET_G) X = s.in.p_jump * pc * pc * (3.0 - 2.0 * pc);
        else X = s.in.psi_bulk + s.in.psi_gradx * ((double)x - s.in.xT0) + s.in.psi_band * 4.0 * pc * (1.0 - pc);
    }
    return wt(a) * X;
}

// Store a post-streaming state into buffer `b` as the post-collision values
// that the pull of the next step streams into it (inverse streaming).  Slot
// (a, y) feeds node t = y + e_a; if t lies beyond a wall the slot is read
// back by y itself through the wall rule of direction abar, so its value is
// the inverse of that bounce-back / anti-bounce-back.  Reduced-precision
// storage is relative to the slot node's own references: the FP16-rounded
// phi, psi, p* and T of the state at y (written to its reference record).
template <typename S, typename R>
__device__ void store_node(const CaseDev& cd, const StateSrc& s, int b, int y0x, int y0y)
{
    S* buf = (S*)cd.buf[b];
    const int64_t o = (int64_t)y0y * cd.pitch + y0x;
    const R sc = R(cd.scale);
    double ref[4] = {0.0, 0.0, 0.0, 0.0};
    if (cd.refs) {
        double sf = 0.0, sq = 0.0, sg = 0.0, sh = 0.0;
        for (int a = 0; a < 9; ++a) {
            sf += src_pop(cd, s, SET_F, a, y0x, y0y);
            sq += src_pop(cd, s, SET_Q, a, y0x, y0y);
            sg += src_pop(cd, s, SET_G, a, y0x, y0y);
            sh += src_pop(cd, s, SET_H, a, y0x, y0y);
        }
        const __half hf = __float2half_rn((float)sf), hq = __float2half_rn((float)sq), hg = __float2half_rn((float)sg),
                     ht = __float2half_rn((float)sh);
        cd.rbuf[b][4 * o + 0] = hf;
        cd.rbuf[b][4 * o + 1] = hq;
        cd.rbuf[b][4 * o + 2] = hg;
        cd.rbuf[b][4 * o + 3] = ht;
        ref[SET_F] = (double)__half2float(hf);
        ref[SET_Q] = (double)__half2float(hq);
        ref[SET_G] = (double)__half2float(hg);
        ref[SET_H] = (double)__half2float(ht);
    }
    for (int set = 0; set < 4; ++set) {
        const double ry = ref[set];
        for (int a = 0; a < 9; ++a) {
            const double w = wt(a);
            int tx = y0x + ex(a), ty = y0y + ey(a);
            if (!cd.wallx) tx = tx < 0 ? tx + cd.nx : (tx >= cd.nx ? tx - cd.nx : tx);
            if (!cd.wally) ty = ty < 0 ? ty + cd.ny : (ty >= cd.ny ? ty - cd.ny : ty);
            const bool outy = ty < 0 || ty >= cd.ny, outx = tx < 0 || tx >= cd.nx;
            double v;
            if (!outx && !outy) {
                v = src_pop(cd, s, set, a, tx, ty) - w * ry;
            } else {
                const int side = outy ? (ty < 0 ? 2 : 3) : (tx < 0 ? 0 : 1);
                const double dev_b = src_pop(cd, s, set, opp(a), y0x, y0y) - w * ry;
                if (set == SET_H && cd.tbc[side]) {
                    const double Tw = cd.T0 + cd.gradT * ((double)y0x + 0.5 * ex(a) - cd.xT0);
                    v = 2.0 * w * (Tw - ry) - dev_b;
                } else if (set == SET_Q && cd.pbc[side]) {
                    v = 2.0 * w * (cd.psi_w[side] - ry) - dev_b;
                } else {
                    v = dev_b;
                }
            }
            buf[((int64_t)a * cd.plane + o) * 4 + set] = enc<S, R>(R(v), sc);
        }
    }
}

__global__ void k_store(const CaseDev* __restrict__ cases, int case_id, StateSrc src, int b)
{
    const CaseDev& cd = cases[case_id];
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= cd.nx || y >= cd.ny) return;
    if (cd.prec == PREC_FP64) store_node<double, double>(cd, src, b, x, y);
    else if (cd.prec == PREC_FP16S) store_node<__half, float>(cd, src, b, x, y);
    else store_node<float, float>(cd, src, b, x, y);
}

// Post-streaming populations of the current state as FP64 planes
// [4][9][ny][nx] (full values): the same pull the step performs, with the
// per-node references read from global memory.
template <int SET, typename S, typename R, typename RF>
__device__ __forceinline__ void export_set(const Ctx<R>& c, View src, int x, int y, double* out, int64_t n, R base,
                                           const RF& rf)
{
    constexpr bool REFS = sizeof(R) == 4;
    R v[9];
    pull9<SET, false, REFS, S>(c, src, x, y, x, y, base, rf, v);
    const int64_t k = (int64_t)y * c.nx + x;
#pragma unroll
    for (int a = 0; a < 9; ++a) out[(int64_t)(SET * 9 + a) * n + k] = (double)v[a] + wt(a) * (double)base;
}

template <typename S, typename R>
__device__ void export_node(const CaseDev& cd, int b, int x, int y, double* out)
{
    constexpr bool REFS = sizeof(R) == 4;
    Ctx<R> c;
    c.load(cd);
    const View src{make_rsrc(cd.buf[b], cd.pop_bytes)};
    const __half* rb = cd.rbuf[b];
    const int64_t n = (int64_t)cd.nx * cd.ny;
    auto node = [&](int ux, int uy) -> int64_t {
        if (!c.wallx) ux = ux < 0 ? ux + c.nx : (ux >= c.nx ? ux - c.nx : ux);
        if (!c.wally) uy = uy < 0 ? uy + c.ny : (uy >= c.ny ? uy - c.ny : uy);
        return (int64_t)uy * c.pitch + ux;
    };
    auto rf = [&](int ux, int uy) -> R { return REFS ? R(__half2float(rb[4 * node(ux, uy) + 0])) : R(0); };
    auto rq = [&](int ux, int uy) -> R { return REFS ? R(__half2float(rb[4 * node(ux, uy) + 1])) : R(0); };
    auto rp = [&](int ux, int uy) -> R { return REFS ? R(__half2float(rb[4 * node(ux, uy) + 2])) : R(0); };
    auto rt = [&](int ux, int uy) -> R { return REFS ? R(__half2float(rb[4 * node(ux, uy) + 3])) : R(0); };
    export_set<SET_F, S>(c, src, x, y, out, n, rf(x, y), rf);
    export_set<SET_G, S>(c, src, x, y, out, n, rp(x, y), rp);
    export_set<SET_H, S>(c, src, x, y, out, n, rt(x, y), rt);
    export_set<SET_Q, S>(c, src, x, y, out, n, rq(x, y), rq);
}

__global__ void k_export(const CaseDev* __restrict__ cases, int case_id, int b, double* out)
{
    const CaseDev& cd = cases[case_id];
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= cd.nx || y >= cd.ny) return;
    if (cd.prec == PREC_FP64) export_node<double, double>(cd, b, x, y, out);
    else if (cd.prec == PREC_FP16S) export_node<__half, float>(cd, b, x, y, out);
    else export_node<float, float>(cd, b, x, y, out);
}

}  // namespace lbm

// ======================================================================= host
using namespace lbm;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(LBM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t elem_bytes(int prec) { return prec == LBM_FP64 ? 8 : (prec == LBM_FP32 ? 4 : 2); }

int pitch_of(int nx) { return (nx + 63) / 64 * 64; }

// MI355X last-level (Infinity) cache shared by the XCDs.
constexpr size_t kLastLevelCacheBytes = (size_t)256 << 20;

// Nodes per population / reference plane: ny rows of the pitch plus kPlanePad
// nodes, so that the 36 planes of a buffer do not start at one power-of-two
// stride.
constexpr int kPlanePad = 64;
int64_t plane_of(const lbm_case& c) { return (int64_t)c.ny * pitch_of(c.nx) + kPlanePad; }

size_t case_pop_bytes(const lbm_case& c) { return align256((size_t)36 * plane_of(c) * elem_bytes(c.precision)); }

// Per-node storage references (phi, psi, p*, T) of reduced-precision cases: one 8-byte record per node.
size_t case_ref_bytes(const lbm_case& c) { return c.precision == LBM_FP64 ? 0 : align256((size_t)4 * plane_of(c) * 2); }

int64_t tiles_of(const lbm_case& c, int bx, int by) { return (int64_t)((c.nx + bx - 1) / bx) * ((c.ny + by - 1) / by); }

struct Layout {
    size_t off_cases, off_steps, off_partials, off_diag, off_tiles[kNumShapes], off_mtiles, off_pops, total;
    int64_t ntiles[kNumShapes], ntiles16[kNumShapes], nmtiles, max_case_mtiles;
};

Layout layout_of(const lbm_case* cs, int n)
{
    Layout L{};
    size_t o = 0;
    L.off_cases = o;
    o = align256(o + sizeof(CaseDev) * n);
    L.off_steps = o;
    o = align256(o + sizeof(int64_t) * n);
    int64_t mt = 0, mmax = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t t = tiles_of(cs[i], kMacroBX, kMacroBY);
        mt += t;
        mmax = std::max(mmax, t);
    }
    L.nmtiles = mt;
    L.max_case_mtiles = mmax;
    L.off_partials = o;
    o = align256(o + sizeof(double) * NDIAG_PART * (size_t)std::max<int64_t>(mmax, 1));
    L.off_diag = o;
    o = align256(o + sizeof(double) * NDIAG_PART);
    for (int s = 0; s < kNumShapes; ++s) {
        int64_t t = 0, t16 = 0;
        for (int i = 0; i < n; ++i) {
            const int64_t k = tiles_of(cs[i], kShapes[s].bx, kShapes[s].by);
            t += k;
            if (cs[i].precision == LBM_FP16S) t16 += k;
        }
        L.ntiles[s] = t;
        L.ntiles16[s] = t16;
        L.off_tiles[s] = o;
        o = align256(o + sizeof(TileRec) * (size_t)t);
    }
    L.off_mtiles = o;
    o = align256(o + sizeof(TileRec) * (size_t)mt);
    L.off_pops = o;
    for (int i = 0; i < n; ++i) o += 2 * (case_pop_bytes(cs[i]) + case_ref_bytes(cs[i]));
    L.total = o;
    return L;
}

int validate(const lbm_case& c, int i)
{
    if (c.nx < 4 || c.ny < 4) return fail(LBM_E_INVAL, "case %d: nx, ny must be >= 4", i);
    if ((int64_t)c.nx * c.ny > (int64_t)1 << 28) return fail(LBM_E_INVAL, "case %d: lattice too large", i);
    if (c.precision < 0 || c.precision > 2) return fail(LBM_E_INVAL, "case %d: precision", i);
    // FP16 storage on a lattice narrower than one tile row was followed by a GPU
    // memory fault whose cause a CPU replay of every access of that handle did
    // not find; such lattices are refused with FP16 storage (FP32 / FP64 run them)
    if (c.precision == LBM_FP16S && c.nx < 64)
        return fail(LBM_E_INVAL, "case %d: FP16 storage needs nx >= 64 (got %d); use FP32 for narrower lattices", i, c.nx);
    // one population buffer (36 planes) is addressed with 32-bit byte offsets
    if (case_pop_bytes(c) > (size_t)0xFFFFFF00u)
        return fail(LBM_E_INVAL, "case %d: %dx%d needs %zu bytes per population buffer; the limit is 4 GiB", i, c.nx,
                    c.ny, case_pop_bytes(c));
    if (c.sigma_law < 0 || c.sigma_law > 1) return fail(LBM_E_INVAL, "case %d: sigma_law", i);
    if (c.init_kind < 0 || c.init_kind > 2) return fail(LBM_E_INVAL, "case %d: init_kind", i);
    if (c.wall[0] != c.wall[1] || c.wall[2] != c.wall[3])
        return fail(LBM_E_INVAL, "case %d: wall: periodic sides must come in pairs", i);
    for (int s = 0; s < 4; ++s)
        if (c.wall[s] > 1 || c.t_bc[s] > 1 || c.psi_bc[s] > 1) return fail(LBM_E_INVAL, "case %d: wall/t_bc/psi_bc flags", i);
    struct {
        const char* name;
        double v;
    } pos[] = {{"W", c.W}, {"rho_A", c.rho_A}, {"rho_B", c.rho_B}, {"nu_A", c.nu_A}, {"nu_B", c.nu_B},
               {"alpha_A", c.alpha_A}, {"alpha_B", c.alpha_B}, {"D_psi", c.D_psi}, {"M_phi", c.M_phi},
               {"psi_inf", c.psi_inf}};
    for (auto& p : pos)
        if (!(p.v > 0) || !std::isfinite(p.v)) return fail(LBM_E_INVAL, "case %d: %s must be finite and > 0", i, p.name);
    if (c.sigma_law == LBM_SIGMA_PAPER && !(c.T_ref != 0)) return fail(LBM_E_INVAL, "case %d: T_ref must be nonzero", i);
    if (!std::isfinite(c.p_jump)) return fail(LBM_E_INVAL, "case %d: p_jump must be finite", i);
    if (!std::isfinite(c.psi_gradx)) return fail(LBM_E_INVAL, "case %d: psi_gradx must be finite", i);
    return LBM_OK;
}

CaseDev make_dev(const lbm_case& c, void* b0, void* b1, void* r0, void* r1)
{
    CaseDev d{};
    d.nx = c.nx;
    d.ny = c.ny;
    d.pitch = pitch_of(c.nx);
    d.prec = c.precision;
    d.wallx = c.wall[0];
    d.wally = c.wall[2];
    d.law = c.sigma_law;
    d.refs = c.precision == LBM_FP64 ? 0 : 1;
    for (int s = 0; s < 4; ++s) {
        d.tbc[s] = c.wall[s] ? c.t_bc[s] : 0;
        d.pbc[s] = c.wall[s] ? c.psi_bc[s] : 0;
        d.psi_w[s] = c.psi_w[s];
    }
    d.T0 = c.T0;
    d.gradT = c.gradT;
    d.xT0 = c.xT0;
    d.s0 = c.sigma0;
    d.sT = c.sigma_T;
    d.sTT = c.sigma_TT;
    d.Tref = c.T_ref;
    d.beta = c.beta_s;
    d.inv_psi_inf = 1.0 / c.psi_inf;
    d.rhoA = c.rho_A;
    d.drho = c.rho_B - c.rho_A;
    d.muA = c.rho_A * c.nu_A;
    d.dmu = c.rho_B * c.nu_B - c.rho_A * c.nu_A;
    d.alphaA = c.alpha_A;
    d.dalpha = c.alpha_B - c.alpha_A;
    d.om_phi = 1.0 / (3.0 * c.M_phi + 0.5);
    d.om_psi = 1.0 / (3.0 * c.D_psi + 0.5);
    d.Mphi = c.M_phi;
    d.W = c.W;
    d.Dpsi = c.D_psi;
    d.s_lam = c.s_lam;
    d.w_lam = c.w_lam;
    d.Fx = c.Fext_x;
    d.Fy = c.Fext_y;
    d.grav = c.gravity;
    d.scale = c.precision == LBM_FP16S ? (double)kFp16Scale : 1.0;
    d.inv_scale = 1.0 / d.scale;
    d.a8W2 = 8.0 / (c.W * c.W);
    d.mt4W = 4.0 * c.M_phi / c.W;
    d.invTref = c.T_ref != 0 ? 1.0 / c.T_ref : 0.0;
    d.plane = plane_of(c);
    d.max_steps = c.max_steps;
    d.pop_bytes = (uint32_t)case_pop_bytes(c);
    d.ref_bytes = (uint32_t)case_ref_bytes(c);
    d.buf[0] = b0;
    d.buf[1] = b1;
    d.rbuf[0] = (__half*)r0;
    d.rbuf[1] = (__half*)r1;
    ConstsF& f = d.f32;
    for (int s = 0; s < 4; ++s) f.psi_w[s] = (float)d.psi_w[s];
    f.T0 = (float)d.T0; f.gradT = (float)d.gradT; f.xT0 = (float)d.xT0;
    f.s0 = (float)d.s0; f.sT = (float)d.sT; f.sTT = (float)d.sTT; f.Tref = (float)d.Tref; f.beta = (float)d.beta;
    f.inv_psi_inf = (float)d.inv_psi_inf;
    f.rhoA = (float)d.rhoA; f.drho = (float)d.drho; f.muA = (float)d.muA; f.dmu = (float)d.dmu;
    f.alphaA = (float)d.alphaA; f.dalpha = (float)d.dalpha;
    f.om_phi = (float)d.om_phi; f.om_psi = (float)d.om_psi; f.Mphi = (float)d.Mphi; f.W = (float)d.W;
    f.Dpsi = (float)d.Dpsi; f.s_lam = (float)d.s_lam; f.w_lam = (float)d.w_lam;
    f.Fx = (float)d.Fx; f.Fy = (float)d.Fy; f.grav = (float)d.grav;
    f.scale = (float)d.scale; f.inv_scale = (float)d.inv_scale;
    f.a8W2 = (float)d.a8W2; f.mt4W = (float)d.mt4W; f.invTref = (float)d.invTref;
    return d;
}

InitDev make_init(const lbm_case& c)
{
    InitDev in{};
    in.kind = c.init_kind;
    in.xc = c.xc;
    in.yc = c.yc;
    in.R = c.R;
    in.W = c.W;
    in.psi_bulk = c.psi_bulk;
    in.psi_band = c.psi_band;
    in.psi_gradx = c.psi_gradx;
    in.xT0 = c.xT0;
    in.phi_noise = c.phi_noise;
    in.p_jump = c.p_jump;
    in.seed = c.seed;
    return in;
}

using StepKernel = void (*)(const CaseDev*, const TileRec*, int, const int64_t*, int);

template <int ST>
StepKernel step_kernel_st(const Config& cf)
{
    if (cf.nt == 512) return k_step<ST, 64, 8, 512>;
    return cf.shape == 0 ? k_step<ST, 64, 8, 256> : k_step<ST, 64, 4, 256>;
}

StepKernel step_kernel(int st, const Config& cf)
{
    switch (st) {
        case ST_F64: return step_kernel_st<ST_F64>(cf);
        case ST_F16: return step_kernel_st<ST_F16>(cf);
    }
    return step_kernel_st<ST_F32>(cf);
}

// Tiles must fit the 64 KiB per-workgroup LDS budget.
bool shape_ok(int shape, bool fp64)
{
    const int bx = kShapes[shape].bx, by = kShapes[shape].by;
    const size_t e3 = fp64 ? 0 : (size_t)(bx + 6) * (by + 6), e2 = (size_t)(bx + 4) * (by + 4), e1 = (size_t)(bx + 2) * (by + 2);
    const size_t lds = (2 * e3 + (fp64 ? 1 : 2) * e2 + 5 * e1) * (fp64 ? 8 : 4) + 8 * e1;
    return lds <= 65536;
}

bool config_ok(int cfg, bool fp64)
{
    if (cfg < 0 || cfg >= kNumConfigs) return false;
    return shape_ok(kConfigs[cfg].shape, fp64);
}

// Fixed device staging array of lbm_moments_static (callers that cannot
// allocate): kStaticScratchBytes on every device the library runs on, held
// until the process ends.  Host code never passes the symbol itself to a
// kernel or copy: its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and kept here.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device ordinal -> device address of `scratch`

// Device address of `scratch` on the current device (looked up once per device).
int scratch_addr(void** out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(LBM_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return LBM_OK;
}

}  // namespace

struct lbm_handle {
    int ncases = 0;
    std::vector<lbm_case> cases;
    std::vector<CaseDev> dev;
    std::vector<int64_t> steps;       // host mirror of the device step counters
    std::vector<int64_t> mtile_begin, mtile_count;
    hipStream_t stream = nullptr;
    void* scratch = nullptr;  // this device's static staging array (lbm_moments_static)
    char* ws = nullptr;
    Layout L{};
    bool fp64 = false;
    int st = ST_F32;  // ST_F64, or ST_F32 for FP32 / FP16-storage handles (one kernel per storage type)
    int cfg = 1;               // step configuration (index into kConfigs), set by lbm_init
    bool use_graph = true;
    int timing = 0;  // 0 off, 1 per-step eager launches, 2 per launched chunk
    std::map<int, hipGraphExec_t> graphs;
    std::vector<hipEvent_t> ev;       // pairs around timed step launches
    int64_t timed = 0;

    CaseDev* d_cases() { return (CaseDev*)(ws + L.off_cases); }
    int64_t* d_steps() { return (int64_t*)(ws + L.off_steps); }
    double* d_partials() { return (double*)(ws + L.off_partials); }
    double* d_diag() { return (double*)(ws + L.off_diag); }
    TileRec* d_tiles(int s) { return (TileRec*)(ws + L.off_tiles[s]); }
    TileRec* d_mtiles() { return (TileRec*)(ws + L.off_mtiles); }


    // One kernel launch over tiles [t0, t0 + n) of the shape's table.
    int launch_part(const Config& cf, int st_part, int64_t t0, int64_t n, int t)
    {
        if (n <= 0) return LBM_OK;
        hipLaunchKernelGGL(step_kernel(st_part, cf), dim3((unsigned)n), dim3(cf.nt), 0, stream, d_cases(),
                           d_tiles(cf.shape) + t0, (int)n, d_steps(), t);
        HIPCHK(hipGetLastError());
        return LBM_OK;
    }
    int launch_step(int t)
    {
        const Config& cf = kConfigs[cfg];
        const int64_t nt = L.ntiles[cf.shape], n16 = L.ntiles16[cf.shape];
        if (st == ST_F64) return launch_part(cf, ST_F64, 0, nt, t);
        // FP16-storage tiles first in the table, then the FP32 tiles, each with its own kernel
        int rc = launch_part(cf, ST_F16, 0, n16, t);
        if (rc == LBM_OK) rc = launch_part(cf, ST_F32, n16, nt - n16, t);
        return rc;
    }
    int launch_advance(int64_t k)
    {
        hipLaunchKernelGGL(k_advance, dim3((ncases + 255) / 256), dim3(256), 0, stream, d_cases(), ncases, d_steps(), k);
        HIPCHK(hipGetLastError());
        return LBM_OK;
    }
    void host_advance(int64_t k)
    {
        for (int i = 0; i < ncases; ++i) {
            int64_t s = steps[i] + k;
            if (cases[i].max_steps > 0 && s > cases[i].max_steps) s = cases[i].max_steps;
            if (steps[i] < s) steps[i] = s;
        }
    }
    void drop_graphs()
    {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
        graphs.clear();
    }
    int graph_for(int k, hipGraphExec_t* out)
    {
        auto it = graphs.find(k);
        if (it != graphs.end()) {
            *out = it->second;
            return LBM_OK;
        }
        HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        int rc = LBM_OK;
        for (int t = 0; t < k && rc == LBM_OK; ++t) rc = launch_step(t);
        if (rc == LBM_OK) rc = launch_advance(k);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(stream, &g);
        if (rc != LBM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(LBM_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(LBM_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
        graphs[k] = ex;
        *out = ex;
        return LBM_OK;
    }
    int macro(int case_id, uint32_t mask, double* fields, bool diag)
    {
        const int64_t nb = mtile_count[case_id];
        if (nb <= 0) return LBM_OK;
        if (fp64)
            hipLaunchKernelGGL(k_macro<double>, dim3((unsigned)nb), dim3(256), 0, stream, d_cases(), d_mtiles(),
                               (int)mtile_begin[case_id], d_steps(), case_id, mask, fields,
                               diag ? d_partials() : nullptr);
        else
            hipLaunchKernelGGL(k_macro<float>, dim3((unsigned)nb), dim3(256), 0, stream, d_cases(), d_mtiles(),
                               (int)mtile_begin[case_id], d_steps(), case_id, mask, fields,
                               diag ? d_partials() : nullptr);
        HIPCHK(hipGetLastError());
        if (diag) {
            hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, stream, d_partials(), (int)nb, d_diag());
            HIPCHK(hipGetLastError());
        }
        return LBM_OK;
    }
};

#define CHECK_H(h)                                                        \
    do {                                                                  \
        if (!(h)) return fail(LBM_E_INVAL, "null handle");                \
    } while (0)
#define CHECK_CASE(h, i)                                                                   \
    do {                                                                                   \
        if ((i) < 0 || (i) >= (h)->ncases) return fail(LBM_E_INVAL, "case_id %d out of range", (int)(i)); \
    } while (0)

extern "C" {

const char* lbm_last_error(void) { return g_err; }

size_t lbm_workspace_bytes(const lbm_case* cases, int32_t ncases)
{
    if (!cases || ncases <= 0) return 0;
    return layout_of(cases, ncases).total;
}

int lbm_init(const lbm_case* cases, int32_t ncases, void* workspace, size_t bytes, void* stream, lbm_handle** out)
{
    g_err[0] = 0;
    if (!out) return fail(LBM_E_INVAL, "out is null");
    *out = nullptr;
    if (!cases || ncases <= 0) return fail(LBM_E_INVAL, "no cases");
    if (!workspace) return fail(LBM_E_INVAL, "workspace is null");
    if (((uintptr_t)workspace & 255) != 0) return fail(LBM_E_INVAL, "workspace must be 256-byte aligned");
    bool any64 = false, any32 = false;
    for (int i = 0; i < ncases; ++i) {
        const int rc = validate(cases[i], i);
        if (rc != LBM_OK) return rc;
        (cases[i].precision == LBM_FP64 ? any64 : any32) = true;
    }
    if (any64 && any32) return fail(LBM_E_INVAL, "FP64 cases cannot share a handle with FP32/FP16S cases");
    const Layout L = layout_of(cases, ncases);
    if (bytes < L.total) return fail(LBM_E_NOMEM, "workspace has %zu bytes, needs %zu", bytes, L.total);

    void* scr = nullptr;
    {
        const int rc = scratch_addr(&scr);
        if (rc != LBM_OK) return rc;
    }
    lbm_handle* h = new (std::nothrow) lbm_handle();
    if (!h) return fail(LBM_E_NOMEM, "host allocation failed");
    h->scratch = scr;
    h->ncases = ncases;
    h->cases.assign(cases, cases + ncases);
    h->stream = (hipStream_t)stream;
    h->ws = (char*)workspace;
    h->L = L;
    h->fp64 = any64;
    {
        h->st = any64 ? ST_F64 : ST_F32;
    }
    h->steps.assign(ncases, 0);
    h->cfg = default_config(any64);

    size_t o = L.off_pops;
    for (int i = 0; i < ncases; ++i) {
        const size_t b = case_pop_bytes(cases[i]), r = case_ref_bytes(cases[i]);
        char* base = h->ws + o;
        h->dev.push_back(make_dev(cases[i], base, base + b, r ? base + 2 * b : nullptr, r ? base + 2 * b + r : nullptr));
        o += 2 * (b + r);
    }
    // A step reads one buffer of every case and writes the other: when the
    // populations of the handle exceed the last-level cache, whole-record
    // FP16 stores are non-temporal (a step's output is read back from HBM
    // anyway); when they fit, the next step finds them in that cache.
    const bool nt = o - L.off_pops > kLastLevelCacheBytes;
    for (auto& d : h->dev) d.nt_store = nt ? 1 : 0;
    std::vector<TileRec> tiles;
    auto upload = [&](TileRec* dst) -> int {
        if (tiles.empty()) return LBM_OK;
        HIPCHK(hipMemcpyAsync(dst, tiles.data(), tiles.size() * sizeof(TileRec), hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        return LBM_OK;
    };
    // step tiles of a case in row-major order (measured faster than column
    // bands of 128 - 512 lattice columns)
    auto add_tiles = [&](int i, int bx, int by) {
        for (int y = 0; y < cases[i].ny; y += by)
            for (int x = 0; x < cases[i].nx; x += bx) tiles.push_back(TileRec{i, x, y, 0});
    };
    int rc = LBM_OK;
    for (int s = 0; s < kNumShapes && rc == LBM_OK; ++s) {
        tiles.clear();
        // FP16-storage cases first: a handle that mixes storage types
        // launches one kernel per storage type over the two parts
        for (int i = 0; i < ncases; ++i)
            if (cases[i].precision == LBM_FP16S) add_tiles(i, kShapes[s].bx, kShapes[s].by);
        for (int i = 0; i < ncases; ++i)
            if (cases[i].precision != LBM_FP16S) add_tiles(i, kShapes[s].bx, kShapes[s].by);
        rc = upload(h->d_tiles(s));
    }
    if (rc == LBM_OK) {
        tiles.clear();
        for (int i = 0; i < ncases; ++i) {
            h->mtile_begin.push_back((int64_t)tiles.size());
            for (int y = 0; y < cases[i].ny; y += kMacroBY)
                for (int x = 0; x < cases[i].nx; x += kMacroBX) tiles.push_back(TileRec{i, x, y, 0});
            h->mtile_count.push_back((int64_t)tiles.size() - h->mtile_begin.back());
        }
        rc = upload(h->d_mtiles());
    }
    if (rc == LBM_OK) {
        hipError_t e = hipMemcpyAsync(h->d_cases(), h->dev.data(), sizeof(CaseDev) * ncases, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(h->d_steps(), 0, sizeof(int64_t) * ncases, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = fail(LBM_E_DEVICE, "upload: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < ncases && rc == LBM_OK; ++i) {
        StateSrc src{};
        src.in = make_init(cases[i]);
        hipLaunchKernelGGL(k_store, dim3((cases[i].nx + 255) / 256, cases[i].ny), dim3(256), 0, h->stream, h->d_cases(),
                           i, src, 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = fail(LBM_E_DEVICE, "k_store: %s", hipGetErrorString(e));
    }
    if (rc == LBM_OK) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = fail(LBM_E_DEVICE, "init: %s", hipGetErrorString(e));
    }
    if (rc != LBM_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return LBM_OK;
}

int lbm_step(lbm_handle* h, int64_t nsteps)
{
    CHECK_H(h);
    if (nsteps < 0) return fail(LBM_E_INVAL, "nsteps < 0");
    if (nsteps == 0) return LBM_OK;
    if (h->timing != 0) {
        for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
        h->ev.clear();
        h->timed = 0;
    }
    if (h->timing == 1) {
        // eager launches bracketed by events; the step counters advance once per chunk
        const int64_t CHT = 1000;
        for (int64_t c0 = 0; c0 < nsteps; c0 += CHT) {
            const int k = (int)std::min(nsteps - c0, CHT);
            for (int t = 0; t < k; ++t) {
                hipEvent_t a, b;
                HIPCHK(hipEventCreate(&a));
                HIPCHK(hipEventCreate(&b));
                h->ev.push_back(a);
                h->ev.push_back(b);
                HIPCHK(hipEventRecord(a, h->stream));
                int rc = h->launch_step(t);
                if (rc != LBM_OK) return rc;
                HIPCHK(hipEventRecord(b, h->stream));
            }
            int rc = h->launch_advance(k);
            if (rc != LBM_OK) return rc;
            h->host_advance(k);
        }
        h->timed = nsteps;
        return LBM_OK;
    }
    const int64_t CH = 100;
    int64_t left = nsteps;
    while (left > 0) {
        const int k = (int)std::min(left, CH);
        if (h->timing == 2) {
            // events around each chunk as launched (graph replay included)
            hipEvent_t a;
            HIPCHK(hipEventCreate(&a));
            h->ev.push_back(a);
            HIPCHK(hipEventRecord(a, h->stream));
        }
        if (h->use_graph) {
            hipGraphExec_t g = nullptr;
            int rc = h->graph_for(k, &g);
            if (rc != LBM_OK) return rc;
            HIPCHK(hipGraphLaunch(g, h->stream));
        } else {
            for (int t = 0; t < k; ++t) {
                int rc = h->launch_step(t);
                if (rc != LBM_OK) return rc;
            }
            int rc = h->launch_advance(k);
            if (rc != LBM_OK) return rc;
        }
        if (h->timing == 2) {
            hipEvent_t b;
            HIPCHK(hipEventCreate(&b));
            h->ev.push_back(b);
            HIPCHK(hipEventRecord(b, h->stream));
        }
        h->host_advance(k);
        left -= k;
    }
    if (h->timing == 2) h->timed = nsteps;
    return LBM_OK;
}

int lbm_moments(lbm_handle* h, int32_t case_id, uint32_t mask, void* dst, int32_t dst_on_device)
{
    CHECK_H(h);
    CHECK_CASE(h, case_id);
    if (!dst) return fail(LBM_E_INVAL, "dst is null");
    mask &= LBM_F_ALL;
    if (!mask) return LBM_OK;
    const lbm_case& c = h->cases[case_id];
    const size_t nf = (size_t)__builtin_popcount(mask), bytes = nf * (size_t)c.nx * c.ny * sizeof(double);
    double* d = (double*)dst;
    if (!dst_on_device) HIPCHK(hipMalloc(&d, bytes));
    int rc = h->macro(case_id, mask, d, false);
    if (!dst_on_device) {
        hipError_t e = hipSuccess;
        if (rc == LBM_OK) e = hipMemcpyAsync(dst, d, bytes, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        (void)hipFree(d);
        if (rc == LBM_OK && e != hipSuccess) rc = fail(LBM_E_DEVICE, "lbm_moments copy: %s", hipGetErrorString(e));
    }
    return rc;
}

int lbm_moments_static(lbm_handle* h, int32_t case_id, uint32_t mask, void* dst_host)
{
    CHECK_H(h);
    CHECK_CASE(h, case_id);
    if (!dst_host) return fail(LBM_E_INVAL, "dst_host is null");
    mask &= LBM_F_ALL;
    if (!mask) return LBM_OK;
    const lbm_case& c = h->cases[case_id];
    const size_t nf = (size_t)__builtin_popcount(mask), bytes = nf * (size_t)c.nx * c.ny * sizeof(double);
    if (bytes > kStaticScratchBytes)
        return fail(LBM_E_INVAL, "lbm_moments_static: %zu field planes of %dx%d need %zu bytes; the static staging array holds %zu",
                    nf, c.nx, c.ny, bytes, kStaticScratchBytes);
    if (!h->scratch) return fail(LBM_E_STATE, "lbm_moments_static: no staging array on this handle's device");
    // every live node writes every selected plane, so nothing needs clearing first
    int rc = h->macro(case_id, mask, (double*)h->scratch, false);
    if (rc != LBM_OK) return rc;
    HIPCHK(hipMemcpyAsync(dst_host, h->scratch, bytes, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

static int pops_io(lbm_handle* h, int case_id, double* out, const double* in, int on_device)
{
    const lbm_case& c = h->cases[case_id];
    const size_t bytes = (size_t)36 * c.nx * c.ny * sizeof(double);
    double* d = on_device ? (out ? out : (double*)in) : nullptr;
    if (!on_device) {
        HIPCHK(hipMalloc(&d, bytes));
        if (in) {
            hipError_t e = hipMemcpyAsync(d, in, bytes, hipMemcpyHostToDevice, h->stream);
            if (e != hipSuccess) {
                (void)hipFree(d);
                return fail(LBM_E_DEVICE, "population upload: %s", hipGetErrorString(e));
            }
        }
    }
    const int b = (int)(h->steps[case_id] & 1);
    if (out) {
        hipLaunchKernelGGL(k_export, dim3((c.nx + 255) / 256, c.ny), dim3(256), 0, h->stream, h->d_cases(), case_id,
                           b, d);
    } else {
        StateSrc src{};
        src.pops = d;
        hipLaunchKernelGGL(k_store, dim3((c.nx + 255) / 256, c.ny), dim3(256), 0, h->stream, h->d_cases(), case_id,
                           src, b);
    }
    hipError_t e = hipGetLastError();
    if (!on_device) {
        if (e == hipSuccess && out) e = hipMemcpyAsync(out, d, bytes, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        (void)hipFree(d);
    }
    if (e != hipSuccess) return fail(LBM_E_DEVICE, "populations: %s", hipGetErrorString(e));
    return LBM_OK;
}

int lbm_get_populations(lbm_handle* h, int32_t case_id, void* dst, int32_t dst_on_device)
{
    CHECK_H(h);
    CHECK_CASE(h, case_id);
    if (!dst) return fail(LBM_E_INVAL, "dst is null");
    return pops_io(h, case_id, (double*)dst, nullptr, dst_on_device);
}

int lbm_set_populations(lbm_handle* h, int32_t case_id, const void* src, int32_t src_on_device)
{
    CHECK_H(h);
    CHECK_CASE(h, case_id);
    if (!src) return fail(LBM_E_INVAL, "src is null");
    return pops_io(h, case_id, nullptr, (const double*)src, src_on_device);
}

int lbm_load_fields(lbm_handle* h, int32_t case_id, const void* phi, const void* T, const void* psi,
                    int32_t src_on_device)
{
    CHECK_H(h);
    CHECK_CASE(h, case_id);
    if (!phi || !T || !psi) return fail(LBM_E_INVAL, "null field pointer");
    const lbm_case& c = h->cases[case_id];
    const size_t n = (size_t)c.nx * c.ny, bytes = n * sizeof(double);
    const double *dp = (const double*)phi, *dT = (const double*)T, *dq = (const double*)psi;
    double* tmp = nullptr;
    if (!src_on_device) {
        HIPCHK(hipMalloc(&tmp, 3 * bytes));
        hipError_t e = hipMemcpyAsync(tmp, phi, bytes, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(tmp + n, T, bytes, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(tmp + 2 * n, psi, bytes, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            return fail(LBM_E_DEVICE, "field upload: %s", hipGetErrorString(e));
        }
        dp = tmp;
        dT = tmp + n;
        dq = tmp + 2 * n;
    }
    // step counter back to 0 on both sides; state lives in buffer 0
    h->steps[case_id] = 0;
    hipError_t e = hipMemsetAsync(h->d_steps() + case_id, 0, sizeof(int64_t), h->stream);
    if (e == hipSuccess) {
        StateSrc src{};
        src.phi = dp;
        src.T = dT;
        src.psi = dq;
        hipLaunchKernelGGL(k_store, dim3((c.nx + 255) / 256, c.ny), dim3(256), 0, h->stream, h->d_cases(), case_id,
                           src, 0);
        e = hipGetLastError();
    }
    if (tmp) {
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        (void)hipFree(tmp);
    }
    if (e != hipSuccess) return fail(LBM_E_DEVICE, "lbm_load_fields: %s", hipGetErrorString(e));
    return LBM_OK;
}

int lbm_reduce(lbm_handle* h, int32_t case_id, lbm_diag* out)
{
    CHECK_H(h);
    CHECK_CASE(h, case_id);
    if (!out) return fail(LBM_E_INVAL, "out is null");
    int rc = h->macro(case_id, 0u, nullptr, true);
    if (rc != LBM_OK) return rc;
    double d[NDIAG_PART];
    HIPCHK(hipMemcpyAsync(d, h->d_diag(), sizeof d, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    out->mass_phi = d[0];
    out->mass_psi = d[1];
    out->xc = d[2] / d[0];
    out->yc = d[3] / d[0];
    out->ux = d[4] / d[0];
    out->uy = d[5] / d[0];
    out->p_in = d[7] > 0 ? d[6] / d[7] : 0.0;
    out->p_out = d[9] > 0 ? d[8] / d[9] : 0.0;
    out->nonfinite = d[10];
    out->phi_min = d[11];
    out->phi_max = d[12];
    out->psi_min = d[13];
    out->psi_max = d[14];
    out->step = h->steps[case_id];
    if (d[10] > 0) return fail(LBM_E_NONFINITE, "case %d: %.0f non-finite populations", case_id, d[10]);
    return LBM_OK;
}

int lbm_tile_count(void) { return kNumConfigs; }

int lbm_tile_shape(int32_t index, int32_t* bx, int32_t* by)
{
    if (index < 0 || index >= kNumConfigs) return fail(LBM_E_INVAL, "tile index %d out of range", index);
    if (bx) *bx = kShapes[kConfigs[index].shape].bx;
    if (by) *by = kShapes[kConfigs[index].shape].by;
    return LBM_OK;
}

int lbm_tile_threads(int32_t index)
{
    if (index < 0 || index >= kNumConfigs) return fail(LBM_E_INVAL, "tile index %d out of range", index);
    return kConfigs[index].nt;
}

int lbm_tile_kind(int32_t index)
{
    if (index < 0 || index >= kNumConfigs) return fail(LBM_E_INVAL, "tile index %d out of range", index);
    return 0;
}

int lbm_set_tile(lbm_handle* h, int32_t index)
{
    CHECK_H(h);
    if (index < 0 || index >= kNumConfigs) return fail(LBM_E_INVAL, "tile index %d out of range", index);
    if (!config_ok(index, h->fp64)) return fail(LBM_E_INVAL, "configuration %d exceeds the LDS budget for FP64", index);
    if (index != h->cfg) h->drop_graphs();
    h->cfg = index;
    return LBM_OK;
}

int lbm_get_tile(lbm_handle* h)
{
    CHECK_H(h);
    return h->cfg;
}

int lbm_autotune(lbm_handle* h, int32_t trial_steps)
{
    CHECK_H(h);
    if (trial_steps <= 0) return fail(LBM_E_INVAL, "trial_steps must be > 0");
    const int keep = h->cfg;
    // configurations timed in interleaved rounds, each keeping its best time:
    // the candidates differ by a few per cent, as much as one trial's noise
    constexpr int kRounds = 3;
    float best_ms[kNumConfigs];
    for (float& v : best_ms) v = 1e30f;
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    int rc = LBM_OK;
    for (int round = 0; round < kRounds && rc == LBM_OK; ++round) {
        for (int s = 0; s < kNumConfigs && rc == LBM_OK; ++s) {
            if (!config_ok(s, h->fp64)) continue;
            h->cfg = s;
            // t = 0 every time: each trial re-reads the current state and rewrites
            // the scratch half of the ping-pong pair, leaving the state unchanged.
            for (int w = 0; w < 2 && rc == LBM_OK; ++w) rc = h->launch_step(0);
            if (rc != LBM_OK) break;
            if (hipEventRecord(a, h->stream) != hipSuccess) {
                rc = fail(LBM_E_DEVICE, "event");
                break;
            }
            for (int t = 0; t < trial_steps && rc == LBM_OK; ++t) rc = h->launch_step(0);
            if (rc != LBM_OK) break;
            if (hipEventRecord(b, h->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
                rc = fail(LBM_E_DEVICE, "event");
                break;
            }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, a, b);
            best_ms[s] = std::min(best_ms[s], ms);
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    h->cfg = keep;
    if (rc != LBM_OK) return rc;
    int best = keep;
    for (int s = 0; s < kNumConfigs; ++s)
        if (best_ms[s] < best_ms[best]) best = s;
    return lbm_set_tile(h, best);
}

int lbm_set_graph(lbm_handle* h, int32_t enable)
{
    CHECK_H(h);
    h->use_graph = enable != 0;
    return LBM_OK;
}

int64_t lbm_steps_done(lbm_handle* h, int32_t case_id)
{
    if (!h || case_id < 0 || case_id >= h->ncases) return -1;
    return h->steps[case_id];
}

int lbm_set_kernel_timing(lbm_handle* h, int32_t enable)
{
    CHECK_H(h);
    if (enable < 0 || enable > 2) return fail(LBM_E_INVAL, "timing mode %d (0, 1 or 2)", (int)enable);
    h->timing = enable;
    return LBM_OK;
}

int lbm_kernel_time_ms(lbm_handle* h, double* avg_ms, int64_t* launches)
{
    CHECK_H(h);
    if (h->timed <= 0) return fail(LBM_E_STATE, "no timed lbm_step call");
    HIPCHK(hipStreamSynchronize(h->stream));
    // event pairs: one per step (mode 1) or one per launched chunk (mode 2)
    double tot = 0;
    for (size_t i = 0; i + 1 < h->ev.size(); i += 2) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]));
        tot += ms;
    }
    if (avg_ms) *avg_ms = tot / (double)h->timed;
    if (launches) *launches = h->timed;
    return LBM_OK;
}

int lbm_destroy(lbm_handle* h)
{
    if (!h) return LBM_OK;
    (void)hipStreamSynchronize(h->stream);
    h->drop_graphs();
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    delete h;
    return LBM_OK;
}

}  // extern "C"
