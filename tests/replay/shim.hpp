// Host shims for replaying the gfx950 device code on the CPU with bounds checks.
#pragma once
#include <barrier>
#include <math.h>
using std::isfinite;
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __restrict__

struct Dim3 { unsigned x = 0, y = 0, z = 0; };
extern thread_local Dim3 threadIdx, blockIdx;
extern Dim3 gridDim, blockDim;
extern std::barrier<>* g_bar;
inline void __syncthreads() { g_bar->arrive_and_wait(); }
template <class T> inline T __shfl_xor(T x, int, int) { return x; }

struct __half { uint16_t b; };
struct __half2 { __half x, y; };
inline float __half2float(__half h) { _Float16 f; std::memcpy(&f, &h.b, 2); return (float)f; }
inline __half __float2half_rn(float f) { _Float16 g = (_Float16)f; __half h; std::memcpy(&h.b, &g, 2); return h; }
inline __half2 __floats2half2_rn(float a, float b) { return __half2{__float2half_rn(a), __float2half_rn(b)}; }
inline __half __ushort_as_half(unsigned short u) { return __half{u}; }
inline unsigned short __half_as_ushort(__half h) { return h.b; }
inline float __frcp_rn(float x) { return 1.0f / x; }

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct ShimRsrc { char* base; uint32_t num; };
struct ShimStats { std::atomic<long> loads{0}, stores{0}, oob{0}, oob_vonly{0}; };
extern ShimStats g_stats;
extern thread_local const char* g_ctx;
void shim_report(const char* what, const ShimRsrc& r, uint32_t v, uint32_t s, unsigned n);

inline ShimRsrc shim_make(void* p, int num) { return ShimRsrc{(char*)p, (uint32_t)num}; }
// Hardware: a raw-buffer access is dropped/zero when voffset (+ inst offset) is out of range;
// the scalar offset is NOT part of that check.  We flag any access whose full byte range
// [v + s, v + s + n) leaves [0, num) -- a real fault risk when only v + s (not v) exceeds num.
inline bool shim_chk(const char* what, const ShimRsrc& r, uint32_t v, uint32_t s, unsigned n)
{
    const uint64_t a = (uint64_t)v + s;
    if (a + n > r.num) { shim_report(what, r, v, s, n); return false; }
    return true;
}
template <class T> inline T shim_ld(const ShimRsrc& r, uint32_t v, uint32_t s)
{
    g_stats.loads++;
    T out{};
    if (r.num == 0) return out;
    if (!shim_chk("load", r, v, s, sizeof(T))) return out;
    std::memcpy(&out, r.base + v + s, sizeof(T));
    return out;
}
template <class T> inline void shim_st(T x, const ShimRsrc& r, uint32_t v, uint32_t s)
{
    g_stats.stores++;
    if (r.num == 0) return;
    if (!shim_chk("store", r, v, s, sizeof(T))) return;
    std::memcpy(r.base + v + s, &x, sizeof(T));
}
#define __builtin_amdgcn_make_buffer_rsrc(p, st, n, f) shim_make((p), (n))
#define __builtin_amdgcn_raw_buffer_load_b16(r, v, s, a) shim_ld<uint16_t>((r), (v), (s))
#define __builtin_amdgcn_raw_buffer_load_b32(r, v, s, a) shim_ld<uint32_t>((r), (v), (s))
#define __builtin_amdgcn_raw_buffer_load_b64(r, v, s, a) shim_ld<u32x2>((r), (v), (s))
#define __builtin_amdgcn_raw_buffer_load_b128(r, v, s, a) shim_ld<u32x4>((r), (v), (s))
#define __builtin_amdgcn_raw_buffer_store_b16(x, r, v, s, a) shim_st<uint16_t>((x), (r), (v), (s))
#define __builtin_amdgcn_raw_buffer_store_b32(x, r, v, s, a) shim_st<uint32_t>((x), (r), (v), (s))
#define __builtin_amdgcn_raw_buffer_store_b64(x, r, v, s, a) shim_st<u32x2>((x), (r), (v), (s))
#define __builtin_amdgcn_raw_buffer_store_b128(x, r, v, s, a) shim_st<u32x4>((x), (r), (v), (s))
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
