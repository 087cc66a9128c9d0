// CPU replay of the library's kernels: the device code itself, compiled for the
// host with the bounds-checking shims of shim.hpp.  For the cases in a file of
// lbm_case structs it runs what the library runs on the GPU -- the initial
// store, N steps of the step kernel of one configuration (FP16-storage tiles
// first, then FP32, as the library launches them), the field export and the
// diagnostic reduction -- and reports every buffer access whose byte range
// leaves its buffer.  Each population and reference buffer is a separate heap
// block of exactly the size the library gives it, so AddressSanitizer also
// sees any plain-pointer overrun, and UBSan's bounds check any LDS index
// outside its array.  Writes the six macroscopic fields of case i to
// <prefix>_<i>.bin.  Exit status 1 when any access was out of range.
#include "lib_host.hpp"
#include <thread>
#include <vector>
#include <fstream>

thread_local Dim3 threadIdx, blockIdx;
Dim3 gridDim, blockDim;
std::barrier<>* g_bar;
ShimStats g_stats;
thread_local const char* g_ctx = "";
static std::mutex g_mu;
static int g_nrep = 0;
static const char* g_kernel = "";
void shim_report(const char* what, const ShimRsrc& r, uint32_t v, uint32_t s, unsigned n)
{
    g_stats.oob++;
    if ((uint64_t)v + n > r.num) g_stats.oob_vonly++;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_nrep++ < 30)
        fprintf(stderr, "OOB %s in %s: block %u,%u thread %u: voff %u soff %u size %u num %u (v alone %s)\n", what,
                g_kernel, blockIdx.x, blockIdx.y, threadIdx.x, v, s, n, r.num,
                (uint64_t)v + n > r.num ? "out" : "IN range: scalar offset carries it out");
}

template <class F>
static void launch(const char* name, unsigned gx, unsigned gy, unsigned block, F body)
{
    g_kernel = name;
    gridDim = {gx, gy, 1};
    blockDim = {block, 1, 1};
    std::barrier<> bar((ptrdiff_t)block);
    g_bar = &bar;
    std::vector<std::thread> th;
    for (unsigned t = 0; t < block; ++t)
        th.emplace_back([&, t] {
            threadIdx = {t, 0, 0};
            for (unsigned by = 0; by < gy; ++by)
                for (unsigned bx = 0; bx < gx; ++bx) {
                    blockIdx = {bx, by, 0};
                    body();
                    bar.arrive_and_wait();
                }
        });
    for (auto& x : th) x.join();
}

int main(int argc, char** argv)
{
    if (argc < 5) { fprintf(stderr, "usage: replay cases.bin nsteps config out_prefix\n"); return 2; }
    std::ifstream f(argv[1], std::ios::binary);
    std::vector<char> raw((std::istreambuf_iterator<char>(f)), {});
    const int n = (int)(raw.size() / sizeof(lbm_case));
    std::vector<lbm_case> cs(n);
    memcpy(cs.data(), raw.data(), n * sizeof(lbm_case));
    const int nsteps = atoi(argv[2]), cfg = atoi(argv[3]);
    const int bx = kShapes[kConfigs[cfg].shape].bx, by = kShapes[kConfigs[cfg].shape].by, nthr = kConfigs[cfg].nt;
    bool any64 = false;
    for (int i = 0; i < n; ++i) {
        if (validate(cs[i], i) != LBM_OK) { fprintf(stderr, "invalid: %s\n", g_err); return 2; }
        any64 |= cs[i].precision == LBM_FP64;
    }
    // buffers: one allocation each, exact size (ASan sees any plain-pointer overrun)
    std::vector<CaseDev> dev;
    uint64_t tot = 0;
    for (int i = 0; i < n; ++i) {
        const size_t b = case_pop_bytes(cs[i]), r = case_ref_bytes(cs[i]);
        void* p0 = calloc(1, b); void* p1 = calloc(1, b);
        void* r0 = r ? calloc(1, r) : nullptr; void* r1 = r ? calloc(1, r) : nullptr;
        dev.push_back(make_dev(cs[i], p0, p1, r0, r1));
        tot += 2 * (b + r);
    }
    for (auto& d : dev) d.nt_store = tot > kLastLevelCacheBytes ? 1 : 0;
    std::vector<TileRec> tiles;
    int64_t n16 = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < n; ++i) {
            if ((cs[i].precision == LBM_FP16S) != (pass == 0)) continue;
            for (int y = 0; y < cs[i].ny; y += by)
                for (int x = 0; x < cs[i].nx; x += bx) tiles.push_back(TileRec{i, x, y, 0});
            if (pass == 0) n16 = (int64_t)tiles.size();
        }
    n16 = 0;
    for (auto& t : tiles) n16 += cs[t.c].precision == LBM_FP16S;
    std::vector<int64_t> steps(n, 0);
    // initial state
    for (int i = 0; i < n; ++i) {
        StateSrc src{};
        src.in = make_init(cs[i]);
        launch("k_store", (cs[i].nx + 255) / 256, cs[i].ny, 256, [&] { k_store(dev.data(), i, src, 0); });
    }
    const int64_t nt = (int64_t)tiles.size();
    for (int s0 = 0; s0 < nsteps; s0 += 100) {
        const int k = std::min(100, nsteps - s0);
        for (int t = 0; t < k; ++t) {
            auto run = [&](const char* nm, int st, int64_t t0, int64_t cnt) {
                if (cnt <= 0) return;
                using K = void (*)(const CaseDev*, const TileRec*, int, const int64_t*, int);
                auto pick = [&](auto stc) -> K {
                    constexpr int ST = decltype(stc)::value;
                    if (nthr == 512) return k_step<ST, 64, 8, 512>;
                    return by == 4 ? k_step<ST, 64, 4, 256> : k_step<ST, 64, 8, 256>;
                };
                const K k = st == ST_F64 ? pick(std::integral_constant<int, ST_F64>{})
                          : st == ST_F16 ? pick(std::integral_constant<int, ST_F16>{})
                                         : pick(std::integral_constant<int, ST_F32>{});
                launch(nm, (unsigned)cnt, 1, (unsigned)nthr, [&] { k(dev.data(), tiles.data() + t0, (int)cnt, steps.data(), t); });
            };
            if (any64) run("k_step<F64>", ST_F64, 0, nt);
            else {
                run("k_step<F16>", ST_F16, 0, n16);
                run("k_step<F32>", ST_F32, n16, nt - n16);
            }
        }
        for (int i = 0; i < n; ++i) {
            int64_t s = steps[i] + k;
            if (cs[i].max_steps > 0 && s > cs[i].max_steps) s = cs[i].max_steps;
            steps[i] = s;
        }
    }
    // export: macro fields and diagnostics (64 x 8 macro tiles), post-streaming populations
    for (int i = 0; i < n; ++i) {
        std::vector<TileRec> mt;
        for (int y = 0; y < cs[i].ny; y += kMacroBY)
            for (int x = 0; x < cs[i].nx; x += kMacroBX) mt.push_back(TileRec{i, x, y, 0});
        const size_t np = (size_t)cs[i].nx * cs[i].ny;
        double* fields = (double*)malloc(6 * np * sizeof(double));
        double* part = (double*)malloc(mt.size() * NDIAG_PART * sizeof(double));
        double diag[NDIAG_PART];
        launch("k_macro", (unsigned)mt.size(), 1, 256, [&] {
            if (any64) k_macro<double>(dev.data(), mt.data(), 0, steps.data(), i, LBM_F_ALL_MACRO, fields, nullptr);
            else k_macro<float>(dev.data(), mt.data(), 0, steps.data(), i, LBM_F_ALL_MACRO, fields, nullptr);
        });
        launch("k_macro(diag)", (unsigned)mt.size(), 1, 256, [&] {
            if (any64) k_macro<double>(dev.data(), mt.data(), 0, steps.data(), i, 0u, nullptr, part);
            else k_macro<float>(dev.data(), mt.data(), 0, steps.data(), i, 0u, nullptr, part);
        });
        launch("k_diag_final", 1, 1, 256, [&] { k_diag_final(part, (int)mt.size(), diag); });
        double* pops = (double*)malloc(36 * np * sizeof(double));
        launch("k_export", (cs[i].nx + 255) / 256, cs[i].ny, 256, [&] { k_export(dev.data(), i, (int)(steps[i] & 1), pops); });
        std::string fn = std::string(argv[4]) + "_" + std::to_string(i) + ".bin";
        FILE* fo = fopen(fn.c_str(), "wb");
        fwrite(fields, sizeof(double), 6 * np, fo);
        fclose(fo);
        free(fields); free(part); free(pops);
    }
    printf("replay: %d case(s), %lld tiles (%lld FP16), %d steps, config %d: loads %ld stores %ld out-of-range %ld (voffset alone out of range: %ld)\n",
           n, (long long)nt, (long long)n16, nsteps, cfg, g_stats.loads.load(), g_stats.stores.load(), g_stats.oob.load(),
           g_stats.oob_vonly.load());
    return g_stats.oob.load() ? 1 : 0;
}
