// common.h -- shared device helpers and host plumbing of librsfof.
//
// Pair arithmetic follows the fixed fp32 recipe of rsfof.h: one periodic
// shift per axis, squares summed as ((x^2 + y^2) + z^2), no contraction.
// The library is compiled with -ffp-contract=off; the helpers below keep
// every rounding step as a separate statement so no fusion can occur.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <mutex>

#include "../../include/rsfof.h"

#define RS_DEV __device__ __forceinline__

namespace rs {

// ---------------------------------------------------------------------------
// fp32 pair arithmetic
// ---------------------------------------------------------------------------

RS_DEV float min_image(float d, float L, float h) {
    // one periodic image shift; identical for (i,j) and (j,i) up to sign
    return d > h ? d - L : (d < -h ? d + L : d);
}

RS_DEV float sum_sq3(float dx, float dy, float dz) {
    float sx = dx * dx;
    float sy = dy * dy;
    float sz = dz * dz;
    float t = sx + sy;
    return t + sz;
}

RS_DEV float pos_d2_wrap(float xi, float yi, float zi, float xj, float yj, float zj,
                         float L, float h) {
    return sum_sq3(min_image(xi - xj, L, h), min_image(yi - yj, L, h),
                   min_image(zi - zj, L, h));
}

RS_DEV float pos_d2_nowrap(float xi, float yi, float zi, float xj, float yj, float zj) {
    return sum_sq3(xi - xj, yi - yj, zi - zj);
}

RS_DEV float metric(float a, float Dx, float c, float Dv) {
    float u = a * Dx;
    float w = c * Dv;
    return u + w;
}

// ---------------------------------------------------------------------------
// lock-free union-find over an int32 parent array.
// Invariant: parent[v] <= v, roots satisfy parent[r] == r.  Hooks always put
// the larger root under the smaller one (CAS on the root), so no cycle can
// form; path halving stores only ancestors, which is benign under races.
//
// Reads are relaxed at workgroup scope, so they are served by the XCD's own
// L2 and may return an older value written from another XCD.  An older value
// of parent[v] is still an ancestor of v (links are never undone and every
// store writes an ancestor), so a walk still ends at a former root, two walks
// ending at the same node still prove one component, and a stale answer only
// costs a redundant test.  Hooking is a CAS at agent scope on the root itself:
// it fails on a stale root and returns the current parent, which is smaller,
// so the retry loop makes progress.  Path-halving stores stay at agent scope.
// ---------------------------------------------------------------------------

RS_DEV int uf_load(const int* p, int v) {
    return __hip_atomic_load(p + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

RS_DEV int uf_find(int* par, int v) {
    int cur = uf_load(par, v);
    if (cur == v) return v;
    int prev = v, next;
    while (cur > (next = uf_load(par, cur))) {
        __hip_atomic_store(par + prev, next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        prev = cur;
        cur = next;
    }
    return cur;
}

// read-only root walk used when flattening: it stores nothing, so parallel
// flatteners cannot overwrite a finished entry with an intermediate ancestor
RS_DEV int uf_root(const int* par, int v) {
    int cur = uf_load(par, v);
    while (cur != v) {
        v = cur;
        cur = uf_load(par, v);
    }
    return v;
}

RS_DEV void uf_unite(int* par, int a, int b) {
    int ra = uf_find(par, a), rb = uf_find(par, b);
    while (ra != rb) {
        if (ra > rb) { int t = ra; ra = rb; rb = t; }
        int old = atomicCAS(par + rb, rb, ra);
        if (old == rb) return;
        rb = uf_find(par, old);
        ra = uf_find(par, ra);
    }
}

// ---------------------------------------------------------------------------
// wave-level aggregation of atomics on clustered keys: lanes holding the same
// key elect a leader, so a run of equal keys costs one atomic, not one per
// lane.  Every lane of the wavefront must call these (ballots).
// ---------------------------------------------------------------------------

RS_DEV uint64_t lanemask_lt() { return (1ull << (threadIdx.x & 63)) - 1ull; }

RS_DEV unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        unsigned lo = (unsigned)__shfl_xor((int)(unsigned)v, o, 64);
        unsigned hi = (unsigned)__shfl_xor((int)(unsigned)(v >> 32), o, 64);
        unsigned long long w = ((unsigned long long)hi << 32) | lo;
        v = w < v ? w : v;
    }
    return v;
}

// exact 128-bit helpers
// ---------------------------------------------------------------------------

typedef __int128 i128;
typedef unsigned __int128 u128;

// Round-to-nearest-even conversion of a signed 128-bit integer to fp64.
RS_DEV double i128_to_f64(i128 v) {
    bool neg = v < 0;
    u128 u = neg ? (u128)0 - (u128)v : (u128)v;
    if (u == 0) return 0.0;
    uint64_t hi = (uint64_t)(u >> 64), lo = (uint64_t)u;
    int nbits = hi ? 128 - __builtin_clzll(hi) : 64 - __builtin_clzll(lo);
    double r;
    if (nbits <= 53) {
        r = (double)lo;                       // exact
    } else {
        int shift = nbits - 53;
        u128 m = u >> shift;
        u128 rem = u & (((u128)1 << shift) - 1);
        u128 half = (u128)1 << (shift - 1);
        if (rem > half || (rem == half && (m & 1))) m += 1;
        if (m == ((u128)1 << 53)) { m >>= 1; shift += 1; }
        r = __builtin_ldexp((double)(uint64_t)m, shift);
    }
    return neg ? -r : r;
}

}  // namespace rs

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

#define RS_HIP(expr)                                                        \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) return rs::hip_status(e_);                    \
    } while (0)

#define RS_TRY(expr)                                                        \
    do {                                                                    \
        int s_ = (expr);                                                    \
        if (s_ != RS_OK) return s_;                                         \
    } while (0)

namespace rs {

inline int hip_status(hipError_t e) {
    return e == hipErrorOutOfMemory ? RS_ENOMEM : RS_EDEVICE;
}

// Grow-only per-device workspaces with a bump allocator.  A call reserves
// the footprint of one phase once, then carves sub-buffers (256-byte
// aligned).  AR_BASE holds either the 3D pass's work space or the 6D pass's
// level-0 tables: both entry points synchronise their stream before they
// return, so the two are never live together and share one allocation (at
// 1024^3 each is about 100 GiB; two would not fit beside the large-node work
// space, and re-allocating them on every call costs seconds).  AR_LARGE and
// AR_TREE are the 6D pass's level pipeline, AR_MLP the proposer network,
// AR_SORT the standalone sort.
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t off = 0;
};

constexpr int N_ARENAS = 5;
constexpr int AR_BASE = 0, AR_LARGE = 1, AR_MLP = 2, AR_SORT = 3, AR_TREE = 4;
// The arenas an API call uses; when a reservation cannot be met, the
// device's other arenas (left by earlier calls of other phases) are
// released and the allocation is tried again.
int arena_call_begin(uint32_t keep_mask);
// Serialises the library's calls on the current device (its workspaces are
// per device): every entry point that uses them holds this lock.
int call_lock(std::unique_lock<std::mutex>* lk);
// device bytes the current call could obtain: free memory plus the arenas it
// does not hold plus those in replace_mask (about to be re-reserved)
int device_budget(uint32_t replace_mask, size_t* bytes);
int arena_release(int which);
int arena_reserve(int which, size_t bytes, Arena** out);   // resets the bump pointer
void* arena_take(Arena* a, size_t bytes);       // NULL if the reservation is exceeded
size_t arena_round(size_t bytes);

template <class T>
inline T* take(Arena* a, size_t count) {
    return static_cast<T*>(arena_take(a, count * sizeof(T)));
}

// small pinned host scratch for reading back counters
int host_scratch(void** out, size_t bytes);

inline unsigned grid_for(int64_t n, int block, int64_t cap = 1 << 20) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Optional per-kernel timing with HIP events recorded on the launching
// stream around instrumented launches (off unless enabled by the caller).
// `units` counts the work items a launch processed (members, particles).
void prof_begin(const char* name, hipStream_t st);
void prof_end(const char* name, hipStream_t st, double units);
// Level 2 of the instrumentation also counts the pair tests of the searches
// (kernels built with counters, slower; for measurement runs only).  After a
// counted launch the caller adds its count with prof_add_count (synchronous).
bool prof_count_pairs();
void prof_add_count(const char* name, double count);

// Tuning table: launch shapes chosen per size bucket by the autotuner.  Every
// value is one of a small compiled set; results are the same for all of them.
enum TuneKnob { TUNE_SMALL_NT_256, TUNE_SMALL_NT_1024, TUNE_SMALL_NT_2048, TUNE_XCD_CHUNK,
                TUNE_N };
int tune_get(TuneKnob k);

// device-wide primitives (prims.hip)
size_t scan_temp_bytes(int64_t n);
int scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, void* temp,
                       int32_t* total_dev, hipStream_t st);
size_t sort_temp_bytes(int64_t n);
int sort_pairs_u64_i32(const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                       int32_t* vout, int64_t n, int bits, void* temp, size_t temp_bytes,
                       hipStream_t st);
int fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);

}  // namespace rs
