// sort.hip -- stable LSD radix sort of (u64 key, i32 value) pairs over the
// low `bits` bits of the key, 8-bit digits, one pass per digit (the last
// pass narrower when `bits` is not a multiple of 8).
//
// Each pass:
//   hist     per-tile digit counts, stored digit-major (cnt[d * ntiles + t])
//   scan     exclusive scan of the counts -> global first slot of every
//            (digit, tile) pair; digit-major order keeps tiles in input order
//            inside a digit, which makes the pass stable
//   scatter  each wavefront ranks a contiguous run of the tile's keys
//            (digit peers by ballots, running per-digit counts in its own LDS
//            row), the four rows are combined into slots, the tile is laid out
//            in digit order in LDS and written back: keys of one digit from
//            one tile land in consecutive global slots, so the writes coalesce
// Passes alternate between the output and a scratch buffer so the last one
// lands in the output; the input is never written.
#include "common.h"

namespace rs {

constexpr int RB_T = 256;              // threads per block (4 wavefronts)
constexpr int RB_I = 8;                // keys per thread
constexpr int RB_TILE = RB_T * RB_I;   // keys per tile
constexpr int RB_D = 256;              // digits per pass (equals RB_T)

__global__ void __launch_bounds__(RB_T)
k_rsort_hist(const uint64_t* __restrict__ keys, int64_t n, int shift, uint32_t dmask, int ntiles,
             int32_t* __restrict__ cnt) {
    __shared__ int32_t h[4][RB_D];
    const int tid = threadIdx.x, w = tid >> 6;
    for (int q = 0; q < 4; q++) h[q][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RB_TILE;
    for (int r = 0; r < RB_I; r++) {
        const int64_t i = base + r * RB_T + tid;
        if (i < n) atomicAdd(&h[w][(int)((keys[i] >> shift) & dmask)], 1);
    }
    __syncthreads();
    cnt[(int64_t)tid * ntiles + blockIdx.x] = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
}

__global__ void __launch_bounds__(RB_T)
k_rsort_scatter(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                uint64_t* __restrict__ kout, int32_t* __restrict__ vout, int64_t n, int shift,
                uint32_t dmask, int ntiles, const int32_t* __restrict__ cnt,
                const int32_t* __restrict__ offs) {
    __shared__ uint64_t sk[RB_TILE];
    __shared__ int32_t sv[RB_TILE];
    __shared__ int32_t dstart[RB_D];   // first tile slot of each digit
    __shared__ int32_t gbase[RB_D];    // global slot of that first tile slot
    __shared__ int32_t wc[4][RB_D];    // per wavefront: keys of each digit (then offsets)
    __shared__ int32_t sc[RB_D];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int t = blockIdx.x;
    const int64_t base = (int64_t)t * RB_TILE;
    const int nt = (int)min<int64_t>(RB_TILE, n - base);

    const int c = cnt[(int64_t)tid * ntiles + t];
    gbase[tid] = offs[(int64_t)tid * ntiles + t];
    for (int q = 0; q < 4; q++) wc[q][tid] = 0;
    sc[tid] = c;
    __syncthreads();
    for (int o = 1; o < RB_D; o <<= 1) {
        const int v = tid >= o ? sc[tid - o] : 0;
        __syncthreads();
        sc[tid] += v;
        __syncthreads();
    }
    dstart[tid] = sc[tid] - c;

    // each wavefront ranks its own contiguous run of RB_I * 64 keys in input
    // order: digit peers by ballots, running per-digit counts in its own LDS row
    uint64_t k[RB_I];
    int32_t v[RB_I];
    int rk[RB_I];
    const int64_t wbase = base + (int64_t)w * RB_I * 64;
#pragma unroll
    for (int r = 0; r < RB_I; r++) {
        const int64_t i = wbase + r * 64 + lane;
        const bool ok = i < n;
        k[r] = ok ? kin[i] : 0;
        v[r] = ok ? vin[i] : 0;
        const int d = (int)((k[r] >> shift) & dmask);
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int below = __popcll(peers & lanemask_lt());
        rk[r] = ok ? wc[w][d] + below : -1;
        __builtin_amdgcn_wave_barrier();
        if (ok && below == 0) wc[w][d] += __popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: slots of wavefront w start after the lower wavefronts' keys
    {
        int o = dstart[tid];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int cq = wc[q][tid];
            wc[q][tid] = o;
            o += cq;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RB_I; r++) {
        if (rk[r] >= 0) {
            const int d = (int)((k[r] >> shift) & dmask);
            const int pos = wc[w][d] + rk[r];
            sk[pos] = k[r];
            sv[pos] = v[r];
        }
    }
    __syncthreads();

    for (int j = tid; j < nt; j += RB_T) {
        const uint64_t kk = sk[j];
        const int d = (int)((kk >> shift) & dmask);
        const int64_t g = (int64_t)gbase[d] + (j - dstart[d]);
        kout[g] = kk;
        vout[g] = sv[j];
    }
}

static int64_t rsort_tiles(int64_t n) { return (n + RB_TILE - 1) / RB_TILE; }

size_t sort_temp_bytes(int64_t n) {
    if (n < 1) n = 1;
    const int64_t nc = RB_D * rsort_tiles(n);
    return arena_round((size_t)n * 8) + arena_round((size_t)n * 4) +
           2 * arena_round((size_t)nc * 4) + arena_round(scan_temp_bytes(nc));
}

int sort_pairs_u64_i32(const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                       int32_t* vout, int64_t n, int bits, void* temp, size_t temp_bytes,
                       hipStream_t st) {
    if (n <= 0) return RS_OK;
    if (n >= ((int64_t)1 << 31)) return RS_EINVAL;
    if (temp_bytes < sort_temp_bytes(n) || !temp) return RS_EINTERNAL;
    if (bits < 1) bits = 1;
    if (bits > 64) bits = 64;
    const int passes = (bits + 7) / 8;
    const int64_t ntiles = rsort_tiles(n);
    const int64_t nc = RB_D * ntiles;
    char* p = static_cast<char*>(temp);
    uint64_t* kalt = reinterpret_cast<uint64_t*>(p);
    p += arena_round((size_t)n * 8);
    int32_t* valt = reinterpret_cast<int32_t*>(p);
    p += arena_round((size_t)n * 4);
    int32_t* cnt = reinterpret_cast<int32_t*>(p);
    p += arena_round((size_t)nc * 4);
    int32_t* offs = reinterpret_cast<int32_t*>(p);
    p += arena_round((size_t)nc * 4);
    void* stemp = p;

    const uint64_t* sk = kin;
    const int32_t* svv = vin;
    for (int pass = 0; pass < passes; pass++) {
        const bool to_out = ((passes - 1 - pass) % 2) == 0;
        uint64_t* dk = to_out ? kout : kalt;
        int32_t* dv = to_out ? vout : valt;
        const int shift = 8 * pass;
        const int db = bits - shift < 8 ? bits - shift : 8;   // digit width of this pass
        const uint32_t dmask = (1u << db) - 1u;
        k_rsort_hist<<<(unsigned)ntiles, RB_T, 0, st>>>(sk, n, shift, dmask, (int)ntiles, cnt);
        RS_HIP(hipGetLastError());
        RS_TRY(scan_exclusive_i32(cnt, offs, nc, stemp, nullptr, st));
        k_rsort_scatter<<<(unsigned)ntiles, RB_T, 0, st>>>(sk, svv, dk, dv, n, shift, dmask,
                                                           (int)ntiles, cnt, offs);
        RS_HIP(hipGetLastError());
        sk = dk;
        svv = dv;
    }
    return RS_OK;
}

}  // namespace rs
