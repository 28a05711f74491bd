// prims.hip -- device-wide building blocks: exclusive scan, key/value sort,
// fills, and the per-device workspace.
#include "phase_common.h"

#include <stdlib.h>
#include <string.h>


#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace rs {

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------

static Arena g_arena[64][N_ARENAS];
static uint32_t g_keep[64];          // arenas the current call holds (never released)
static void* g_host_scratch[64];
static size_t g_host_scratch_bytes[64];

size_t arena_round(size_t bytes) { return (bytes + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// tuning table
// ---------------------------------------------------------------------------

struct TuneDef {
    const char* name;
    int value;              // current value (compiled default until set)
    int allowed[4];         // compiled choices, 0-terminated
};
static TuneDef g_tune[TUNE_N] = {
    {"small_threads_256", 256, {128, 256, 0, 0}},
    {"small_threads_1024", 512, {256, 512, 1024, 0}},
    {"small_threads_2048", 1024, {512, 1024, 0, 0}},
    {"xcd_chunk", 1024, {256, 1024, 4096, 0}},
};

int tune_get(TuneKnob k) { return g_tune[k].value; }

bool use_o32(int64_t nmem) {
    return nmem < O32_LIMIT && !getenv("RS_DEBUG_WIDE_OFFSETS");
}

static int tune_find(const char* name) {
    if (!name) return -1;
    for (int k = 0; k < TUNE_N; k++)
        if (strcmp(name, g_tune[k].name) == 0) return k;
    return -1;
}

static int current_device(int* dev) {
    RS_HIP(hipGetDevice(dev));
    return (*dev < 0 || *dev >= 64) ? RS_EDEVICE : RS_OK;
}

static std::mutex g_call_mu[64];

int call_lock(std::unique_lock<std::mutex>* lk) {
    int dev = 0;
    RS_TRY(current_device(&dev));
    *lk = std::unique_lock<std::mutex>(g_call_mu[dev]);
    return RS_OK;
}

int arena_call_begin(uint32_t keep_mask) {
    int dev = 0;
    RS_TRY(current_device(&dev));
    g_keep[dev] = keep_mask;
    return RS_OK;
}

// releases the device's arenas that the current call does not hold
static int arena_release_idle(int dev) {
    for (int k = 0; k < N_ARENAS; k++) {
        Arena* a = &g_arena[dev][k];
        if ((g_keep[dev] >> k) & 1u) continue;
        if (a->base) {
            RS_HIP(hipFree(a->base));
            a->base = nullptr;
            a->cap = 0;
        }
    }
    return RS_OK;
}

int device_budget(uint32_t replace_mask, size_t* bytes) {
    int dev = 0;
    RS_TRY(current_device(&dev));
    size_t fr = 0, tot = 0;
    RS_HIP(hipMemGetInfo(&fr, &tot));
    for (int k = 0; k < N_ARENAS; k++)
        if (!((g_keep[dev] >> k) & 1u) || ((replace_mask >> k) & 1u)) fr += g_arena[dev][k].cap;
    *bytes = fr;
    return RS_OK;
}

int arena_release(int which) {
    int dev = 0;
    RS_TRY(current_device(&dev));
    if (which < 0 || which >= N_ARENAS) return RS_EDEVICE;
    Arena* a = &g_arena[dev][which];
    if (a->base) {
        RS_HIP(hipFree(a->base));
        a->base = nullptr;
        a->cap = 0;
    }
    return RS_OK;
}

int arena_reserve(int which, size_t bytes, Arena** out) {
    int dev = 0;
    RS_TRY(current_device(&dev));
    if (which < 0 || which >= N_ARENAS) return RS_EDEVICE;
    Arena* a = &g_arena[dev][which];
    if (a->cap < bytes) {
        // test hook: a reservation that needs new device memory fails
        if (getenv("RS_DEBUG_FAIL_ALLOC")) return RS_ENOMEM;
        if (a->base) {
            RS_HIP(hipFree(a->base));
            a->base = nullptr;
            a->cap = 0;
        }
        size_t slack = bytes / 16 < ((size_t)1 << 30) ? bytes / 16 : ((size_t)1 << 30);
        size_t want = arena_round(bytes + slack + (1 << 20));
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            // give back what other phases left behind, then try again
            (void)hipGetLastError();
            RS_TRY(arena_release_idle(dev));
            e = hipMalloc(&p, want);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return RS_ENOMEM;
            }
        }
        a->base = static_cast<char*>(p);
        a->cap = want;
    }
    a->off = 0;
    *out = a;
    return RS_OK;
}

void* arena_take(Arena* a, size_t bytes) {
    size_t b = arena_round(bytes ? bytes : 1);
    if (a->off + b > a->cap) return nullptr;
    void* p = a->base + a->off;
    a->off += b;
    return p;
}

int host_scratch(void** out, size_t bytes) {
    int dev = 0;
    RS_HIP(hipGetDevice(&dev));
    if (g_host_scratch_bytes[dev] < bytes) {
        if (g_host_scratch[dev]) RS_HIP(hipHostFree(g_host_scratch[dev]));
        g_host_scratch[dev] = nullptr;
        g_host_scratch_bytes[dev] = 0;
        size_t want = bytes < 4096 ? 4096 : bytes;
        RS_HIP(hipHostMalloc(&g_host_scratch[dev], want, hipHostMallocDefault));
        g_host_scratch_bytes[dev] = want;
    }
    *out = g_host_scratch[dev];
    return RS_OK;
}

// ---------------------------------------------------------------------------
// kernel timing (HIP events on the launching stream)
// ---------------------------------------------------------------------------

struct ProfRec {
    std::vector<hipEvent_t> start, stop;
    std::vector<double> units;
    double done_ms = 0.0, done_units = 0.0;
    int64_t done_launches = 0;
};

static bool g_prof_on = false;
static bool g_prof_pairs = false;
static std::map<std::string, ProfRec> g_prof;
static std::map<std::string, hipEvent_t> g_prof_open;
static std::mutex g_prof_mu;

void prof_begin(const char* name, hipStream_t st) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, st);
    g_prof_open[name] = e;
}

void prof_end(const char* name, hipStream_t st, double units) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    auto it = g_prof_open.find(name);
    if (it == g_prof_open.end()) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, st);
    ProfRec& r = g_prof[name];
    r.start.push_back(it->second);
    r.stop.push_back(e);
    r.units.push_back(units);
    g_prof_open.erase(it);
}

bool prof_count_pairs() { return g_prof_on && g_prof_pairs; }

void prof_add_count(const char* name, double count) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    ProfRec& r = g_prof[name];
    r.done_launches++;
    r.done_units += count;
}

static void prof_drain(ProfRec& r) {
    for (size_t i = 0; i < r.start.size(); i++) {
        float ms = 0.0f;
        (void)hipEventSynchronize(r.stop[i]);
        if (hipEventElapsedTime(&ms, r.start[i], r.stop[i]) == hipSuccess) r.done_ms += ms;
        r.done_units += r.units[i];
        r.done_launches += 1;
        (void)hipEventDestroy(r.start[i]);
        (void)hipEventDestroy(r.stop[i]);
    }
    r.start.clear();
    r.stop.clear();
    r.units.clear();
}

// ---------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------

__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return RS_OK;
    k_fill_i32<<<grid_for(n, 256, 65536), 256, 0, st>>>(p, v, n);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 (three-phase: tile sums, scan of sums, tile scan)
// ---------------------------------------------------------------------------

constexpr int SCAN_BT = 256;
constexpr int SCAN_IPT = 16;
constexpr int SCAN_TILE = SCAN_BT * SCAN_IPT;

// inclusive block scan of one value per thread; returns the block total
__device__ int32_t block_inclusive_scan(int32_t v, int32_t* lds /* [SCAN_BT/64] */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    if (lane == 63) lds[wave] = v;
    __syncthreads();
    int32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < SCAN_BT / 64; w++) {
        int32_t s = lds[w];
        if (w < wave) before += s;
        total += s;
    }
    __syncthreads();
    lds[SCAN_BT / 64] = total;   // scratch slot for callers that need it
    return v + before;
}

__global__ void __launch_bounds__(SCAN_BT) k_tile_sums(const int32_t* __restrict__ in,
                                                       int32_t* __restrict__ sums, int64_t n) {
    __shared__ int32_t lds[SCAN_BT / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; k++) {
        int64_t i = base + k * SCAN_BT + threadIdx.x;
        if (i < n) s += in[i];
    }
    int32_t inc = block_inclusive_scan(s, lds);
    if (threadIdx.x == SCAN_BT - 1) sums[blockIdx.x] = inc;
}

// blocked scan of one tile; adds the tile offset (or 0); writes the grand
// total when this is the last tile and total != NULL
__global__ void __launch_bounds__(SCAN_BT) k_tile_scan(const int32_t* __restrict__ in,
                                                       int32_t* __restrict__ out,
                                                       const int32_t* __restrict__ offs,
                                                       int64_t n, int32_t* __restrict__ total) {
    __shared__ int32_t lds[SCAN_BT / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int32_t v[SCAN_IPT];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; k++) {
        int64_t i = base + k;
        v[k] = i < n ? in[i] : 0;
        s += v[k];
    }
    int32_t inc = block_inclusive_scan(s, lds);
    int32_t run = inc - s + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < SCAN_IPT; k++) {
        int64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BT - 1) *total = run;
}

size_t scan_temp_bytes(int64_t n) {
    size_t b = 0;
    while (n > SCAN_TILE) {
        n = (n + SCAN_TILE - 1) / SCAN_TILE;
        b += arena_round((size_t)n * sizeof(int32_t));
    }
    return b + 256;
}

int scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, void* temp,
                       int32_t* total_dev, hipStream_t st) {
    if (n <= 0) {
        if (total_dev) RS_HIP(hipMemsetAsync(total_dev, 0, sizeof(int32_t), st));
        return RS_OK;
    }
    if (n <= SCAN_TILE) {
        k_tile_scan<<<1, SCAN_BT, 0, st>>>(in, out, nullptr, n, total_dev);
        RS_HIP(hipGetLastError());
        return RS_OK;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    int32_t* sums = static_cast<int32_t*>(temp);
    char* rest = static_cast<char*>(temp) + arena_round((size_t)nb * sizeof(int32_t));
    k_tile_sums<<<(unsigned)nb, SCAN_BT, 0, st>>>(in, sums, n);
    RS_HIP(hipGetLastError());
    RS_TRY(scan_exclusive_i32(sums, sums, nb, rest, total_dev, st));
    k_tile_scan<<<(unsigned)nb, SCAN_BT, 0, st>>>(in, out, sums, n, nullptr);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

}  // namespace rs

extern "C" {

int rs_tune_set(const char* knob, int value) {
    const int k = rs::tune_find(knob);
    if (k < 0) return RS_EINVAL;
    for (int v : rs::g_tune[k].allowed)
        if (v != 0 && v == value) {
            rs::g_tune[k].value = value;
            return RS_OK;
        }
    return RS_EINVAL;
}

int rs_tune_get(const char* knob, int* value, int32_t* choices, int max_choices) {
    const int k = rs::tune_find(knob);
    if (k < 0 || !value) return RS_EINVAL;
    *value = rs::g_tune[k].value;
    int n = 0;
    for (int v : rs::g_tune[k].allowed)
        if (v != 0) {
            if (choices && n < max_choices) choices[n] = v;
            n++;
        }
    return n;
}

const char* rs_tune_name(int index) {
    return (index >= 0 && index < rs::TUNE_N) ? rs::g_tune[index].name : nullptr;
}

int rs_profile_enable(int on) {
    std::lock_guard<std::mutex> g(rs::g_prof_mu);
    if (!on) {
        for (auto& kv : rs::g_prof) rs::prof_drain(kv.second);
        rs::g_prof.clear();
    }
    rs::g_prof_on = on != 0;
    rs::g_prof_pairs = on == 2;
    return RS_OK;
}

int rs_profile_get(const char* name, double* total_ms, int64_t* launches, double* units) {
    if (!name || !total_ms || !launches || !units) return RS_EINVAL;
    std::lock_guard<std::mutex> g(rs::g_prof_mu);
    auto it = rs::g_prof.find(name);
    if (it == rs::g_prof.end()) {
        *total_ms = 0.0;
        *launches = 0;
        *units = 0.0;
        return RS_OK;
    }
    rs::prof_drain(it->second);
    *total_ms = it->second.done_ms;
    *launches = it->second.done_launches;
    *units = it->second.done_units;
    return RS_OK;
}

}  // extern "C"
