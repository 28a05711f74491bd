// props.hip -- per-node halo properties over a 6D hierarchy (the halo
// properties, inertia tensor among them, that the paper's Summary lists as
// new functions of its code).
//
// A node's members are the particles whose deepest node is the node or one
// of its descendants.  Every property is finalised from exact integer sums
// (quantised positions relative to the node's smallest-index member in the
// nearest periodic image, quantised velocities), so any reduction shape
// gives the same bits.
//
// Flow (one stream):
//   1. check the hierarchy (levels sorted, parents one level up and earlier)
//      and sum each node's children's sizes;
//   2. member layout: every subtree is one contiguous range of records --
//      a level-0 node's range starts at the scan of the level-0 sizes, a
//      child's range is carved from its parent's by an atomic bump (the
//      order of siblings does not matter: the sums are exact), and a node's
//      own particles (deepest node == the node) follow its children;
//   3. records: particles are sorted by deepest node (own radix sort), which
//      ranks them inside their node's own range; each particle's position
//      and velocity then go, as one 24-byte record, to that slot;
//   4. reduce: node ranges are cut into chunks of PR_CH members, one
//      wavefront per chunk, members strided over the lanes (coalesced
//      24-byte records); per-lane integer sums are transposed through LDS
//      and summed per quantity; a one-chunk node is finalised at once, the
//      chunks of a larger node add into 128-bit accumulators that a last
//      kernel finalises.
#include <algorithm>

#include "common.h"

namespace rs {

constexpr int PR_SMALL = 64;      // nodes up to this size: one lane per node
constexpr int PR_CH = 2048;       // members per chunk of a larger node (one wavefront)
constexpr int PR_NQ = 15;         // S1 xyz, T1 xyz, S2 xx yy zz xy xz yz, A xyz
constexpr int PR_ACC = 24;        // 64-bit words per accumulated node

struct PrTree {
    const int32_t *level, *parent, *minidx, *size, *deepest;
    int32_t m, nlev;
};

// levels sorted, a level-0 node has no parent, a deeper node's parent is an
// earlier node one level up; records each level's first node and adds every
// node's size to its parent's child sum
__global__ void k_pr_check(PrTree T, int64_t n, int32_t* __restrict__ lstart,
                           int32_t* __restrict__ childsum, int32_t* __restrict__ err) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= T.m) return;
    const int32_t lv = T.level[r], p = T.parent[r], sz = T.size[r], mi = T.minidx[r];
    bool bad = lv < 0 || lv >= T.nlev || sz < 1 || mi < 0 || (int64_t)mi >= n;
    const int32_t lp = r > 0 ? T.level[r - 1] : -1;
    bad |= lv < lp;
    if (lv == 0) bad |= p != -1;
    else bad |= p < 0 || p >= r || T.level[p] != lv - 1;
    if (bad) {
        atomicOr(err, 2);
        return;
    }
    if (lv != lp)
        for (int32_t l = lp + 1; l <= lv; l++) lstart[l] = r;
    if (lv > 0) atomicAdd(childsum + p, sz);
}

// chunk counts (none for a small node), small-node flags, level-0 sizes, and
// the sum of all node sizes (the members the reduction reads), reduced per
// block before one 64-bit atomic
__global__ void __launch_bounds__(256)
k_pr_prep(PrTree T, const int32_t* __restrict__ childsum, int32_t* __restrict__ nch,
          int32_t* __restrict__ small, int32_t* __restrict__ lvl0,
          unsigned long long* __restrict__ members,
          int32_t* __restrict__ err) {
    __shared__ unsigned long long part[4];
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long mine = 0;
    if (r < T.m) {
        const int32_t sz = T.size[r];
        if (childsum[r] > sz) atomicOr(err, 2);
        nch[r] = sz <= PR_SMALL ? 0 : (sz + PR_CH - 1) / PR_CH;
        small[r] = sz <= PR_SMALL ? 1 : 0;
        lvl0[r] = T.level[r] == 0 ? sz : 0;
        mine = (unsigned long long)sz;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mine += (unsigned long long)__shfl_xor((long long)mine, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long b = part[0] + part[1] + part[2] + part[3];
        if (b) atomicAdd(members, b);
    }
}

// offsets of the nodes of level l (grid-stride over the level's range)
__global__ void k_pr_offsets(PrTree T, int32_t l, const int32_t* __restrict__ lstart,
                             int32_t* __restrict__ off, int32_t* __restrict__ cfill) {
    const int32_t b = lstart[l], e = lstart[l + 1];
    for (int32_t r = b + blockIdx.x * blockDim.x + threadIdx.x; r < e;
         r += gridDim.x * blockDim.x) {
        const int32_t p = T.parent[r];
        off[r] = off[p] + atomicAdd(cfill + p, T.size[r]);
    }
}

// Own ranges by sorting: particles are sorted by deepest node (stable radix
// sort; particles outside every node sort last), so the particles of one
// node form one run of the sorted order, in the order of the node indices.
// A particle at sorted position s in node d's run goes to slot
// off[d] + childsum[d] + (s - ownscan[d]), ownscan being the exclusive scan
// of the own counts.  Each run must start at ownscan[d] and hold exactly
// own[d] particles, else the hierarchy is inconsistent (with slot_of NULL
// only that is checked).
__global__ void k_pr_keys(const float* __restrict__ x, const float* __restrict__ y,
                          const float* __restrict__ z, const float* __restrict__ vx,
                          const float* __restrict__ vy, const float* __restrict__ vz,
                          int64_t n, float L, PrTree T, uint64_t* __restrict__ keys,
                          int32_t* __restrict__ idx, int32_t* __restrict__ err) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool bad = !(x[i] >= 0.0f && x[i] < L) || !(y[i] >= 0.0f && y[i] < L) ||
               !(z[i] >= 0.0f && z[i] < L);
    bad |= !(fabsf(vx[i]) < 1048576.0f) || !(fabsf(vy[i]) < 1048576.0f) ||
           !(fabsf(vz[i]) < 1048576.0f);
    if (bad) atomicOr(err, 1);
    int32_t d = T.deepest[i];
    if (d < -1 || d >= T.m) {
        atomicOr(err, 2);
        d = -1;
    }
    keys[i] = d < 0 ? (uint64_t)T.m : (uint64_t)d;
    idx[i] = (int32_t)i;
}

__global__ void k_pr_own(PrTree T, const int32_t* __restrict__ childsum,
                         int32_t* __restrict__ own) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < T.m) own[r] = T.size[r] - childsum[r];
}

__global__ void k_pr_slots(int64_t n, PrTree T, const uint64_t* __restrict__ skey,
                           const int32_t* __restrict__ perm, const int32_t* __restrict__ off,
                           const int32_t* __restrict__ childsum,
                           const int32_t* __restrict__ own, const int32_t* __restrict__ ownscan,
                           int32_t* __restrict__ slot_of, int32_t* __restrict__ err) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t k = skey[s];
    if (k >= (uint64_t)T.m) return;
    const int32_t d = (int32_t)k;
    const int64_t rank = s - ownscan[d];
    const bool first = s == 0 || skey[s - 1] != k;
    const bool last = s + 1 == n || skey[s + 1] != k;
    if (rank < 0 || rank >= own[d] || (first && rank != 0) || (last && rank + 1 != own[d])) {
        atomicOr(err, 2);
        return;
    }
    if (slot_of) slot_of[perm[s]] = off[d] + childsum[d] + (int32_t)rank;
}

__global__ void k_pr_place(const float* __restrict__ x, const float* __restrict__ y,
                           const float* __restrict__ z, const float* __restrict__ vx,
                           const float* __restrict__ vy, const float* __restrict__ vz,
                           int64_t n, PrTree T, const int32_t* __restrict__ slot_of,
                           float2* __restrict__ rec) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t slot = slot_of[i];       // -1: outside every node, or inconsistent
    if (slot < 0 || (int64_t)slot >= n) return;
    const int64_t s = 3 * (int64_t)slot;
    rec[s] = make_float2(x[i], y[i]);
    rec[s + 1] = make_float2(z[i], vx[i]);
    rec[s + 2] = make_float2(vy[i], vz[i]);
}

// quantised position (x < 2048, so x * 2^20 is exact in fp32 and below 2^31)
RS_DEV int32_t pr_qpos(float v) { return (int32_t)rintf(v * 1048576.0f); }
RS_DEV int32_t pr_qvel(float v) { return (int32_t)rintf(v * 1024.0f); }

// one property of a node from its 15 exact sums
RS_DEV float pr_output(int q, const i128* t, int32_t N, const int32_t* qref, float L) {
    const double nn = (double)N * (double)N;
    if (q < 3) {
        double u = ((double)qref[q] + (double)(int64_t)t[q] / (double)N) * 9.5367431640625e-07;
        if (u < 0.0) u += (double)L;
        else if (u >= (double)L) u -= (double)L;
        const float c = (float)u;
        return c >= L ? 0.0f : c;
    }
    if (q < 6) return (float)(((double)(int64_t)t[q] / (double)N) * 9.765625e-4);
    if (q < 12) {
        const int a = q < 9 ? q - 6 : (q == 11 ? 1 : 0);
        const int b = q < 9 ? q - 6 : (q == 9 ? 1 : 2);
        const i128 cm = (i128)N * t[q] - t[a] * t[b];
        return (float)((i128_to_f64(cm) / nn) * 9.094947017729282e-13);
    }
    const int a = q - 12, b = (a + 1) % 3, c = (a + 2) % 3;
    const i128 jn = (i128)N * t[q] - (t[b] * t[3 + c] - t[c] * t[3 + b]);
    return (float)((i128_to_f64(jn) / nn) * 9.313225746154785e-10);
}

// lists of the small nodes and of the chunks of the others
__global__ void k_pr_lists(PrTree T, const int32_t* __restrict__ nch,
                           const int32_t* __restrict__ small, const int32_t* __restrict__ soff,
                           const int32_t* __restrict__ coff, int32_t* __restrict__ slist,
                           int32_t* __restrict__ items) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= T.m) return;
    if (small[r]) {
        slist[soff[r]] = r;
    } else {
        const int32_t b = coff[r];
        for (int32_t c = 0; c < nch[r]; c++) items[b + c] = r;
    }
}

struct PrAcc {
    int64_t s[6];      // S1 xyz, T1 xyz
    i128 w[9];         // S2 xx yy zz xy xz yz, A xyz
};

RS_DEV void pr_zero(PrAcc& a) {
    for (int q = 0; q < 6; q++) a.s[q] = 0;
    for (int q = 0; q < 9; q++) a.w[q] = 0;
}

// add one member record (three float2: x y | z vx | vy vz)
RS_DEV void pr_add(PrAcc& a, float2 r0, float2 r1, float2 r2, const int32_t* qref,
                   int32_t LQh, int32_t LQi, int32_t LQc) {
    const float pv[3] = {r0.x, r0.y, r1.x};
    int32_t d[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        int32_t v = pr_qpos(pv[k]) - qref[k];
        // 2v > LQ  <=>  v > floor(LQ/2);  2v <= -LQ  <=>  v <= -ceil(LQ/2)
        if (v > LQh) v -= LQi;
        else if (v <= -LQc) v += LQi;
        d[k] = v;
    }
    const int32_t w[3] = {pr_qvel(r1.y), pr_qvel(r2.x), pr_qvel(r2.y)};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        a.s[k] += d[k];
        a.s[3 + k] += w[k];
    }
    a.w[0] += (i128)((int64_t)d[0] * d[0]);
    a.w[1] += (i128)((int64_t)d[1] * d[1]);
    a.w[2] += (i128)((int64_t)d[2] * d[2]);
    a.w[3] += (i128)((int64_t)d[0] * d[1]);
    a.w[4] += (i128)((int64_t)d[0] * d[2]);
    a.w[5] += (i128)((int64_t)d[1] * d[2]);
    a.w[6] += (i128)((int64_t)d[1] * w[2] - (int64_t)d[2] * w[1]);
    a.w[7] += (i128)((int64_t)d[2] * w[0] - (int64_t)d[0] * w[2]);
    a.w[8] += (i128)((int64_t)d[0] * w[1] - (int64_t)d[1] * w[0]);
}

struct PrFrame {
    int32_t LQh, LQi, LQc;   // floor(LQ/2), LQ, ceil(LQ/2)
    float L;
};

RS_DEV void pr_ref(const float* __restrict__ x, const float* __restrict__ y,
                   const float* __restrict__ z, int32_t ref, int32_t* qref) {
    qref[0] = pr_qpos(x[ref]);
    qref[1] = pr_qpos(y[ref]);
    qref[2] = pr_qpos(z[ref]);
}

// small nodes: one lane per node, its records read in order
__global__ void __launch_bounds__(256)
k_pr_small(const float* __restrict__ x, const float* __restrict__ y,
           const float* __restrict__ z, int32_t ns, const int32_t* __restrict__ slist,
           PrTree T, PrFrame F, const int32_t* __restrict__ off,
           const float2* __restrict__ rec, float* __restrict__ props) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    const int32_t r = slist[t];
    const int32_t N = T.size[r];
    int32_t qref[3];
    pr_ref(x, y, z, T.minidx[r], qref);
    PrAcc a;
    pr_zero(a);
    const float2* b = rec + 3 * (int64_t)off[r];
    for (int32_t k = 0; k < N; k++)
        pr_add(a, b[3 * k], b[3 * k + 1], b[3 * k + 2], qref, F.LQh, F.LQi, F.LQc);
    i128 tot[PR_NQ];
    for (int q = 0; q < 6; q++) tot[q] = (i128)a.s[q];
    for (int q = 0; q < 9; q++) tot[6 + q] = a.w[q];
    for (int q = 0; q < PR_NQ; q++) props[(int64_t)q * T.m + r] = pr_output(q, tot, N, qref, F.L);
}

RS_DEV uint64_t pr_xor64(uint64_t v, int mask) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, mask, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), mask, 64);
    return ((uint64_t)hi << 32) | lo;
}

// chunks of the larger nodes: one wavefront per chunk, members strided over
// the lanes; two exchange steps leave 16 partial rows, summed per quantity
// through LDS
__global__ void __launch_bounds__(64)
k_pr_large(const float* __restrict__ x, const float* __restrict__ y,
           const float* __restrict__ z, int32_t total, const int32_t* __restrict__ items,
           PrTree T, PrFrame F, const int32_t* __restrict__ off,
           const int32_t* __restrict__ chunk_off, const int32_t* __restrict__ nch,
           const float2* __restrict__ rec, unsigned long long* __restrict__ acc,
           float* __restrict__ props) {
    __shared__ u128 lds[16 + 1][PR_NQ];
    const int lane = threadIdx.x;
    for (int32_t it = blockIdx.x; it < total; it += gridDim.x) {
        const int32_t r = items[it];
        const int32_t c = it - chunk_off[r];
        const int32_t N = T.size[r];
        const int32_t cnt = min(PR_CH, N - c * PR_CH);
        int32_t qref[3];
        pr_ref(x, y, z, T.minidx[r], qref);
        PrAcc a;
        pr_zero(a);
        const float2* b = rec + 3 * ((int64_t)off[r] + (int64_t)c * PR_CH);
#pragma unroll 4
        for (int32_t t = lane; t < cnt; t += 64)
            pr_add(a, b[3 * t], b[3 * t + 1], b[3 * t + 2], qref, F.LQh, F.LQi, F.LQc);
#pragma unroll
        for (int msk = 32; msk >= 16; msk >>= 1) {
#pragma unroll
            for (int q = 0; q < 6; q++) a.s[q] += (int64_t)pr_xor64((uint64_t)a.s[q], msk);
#pragma unroll
            for (int q = 0; q < 9; q++) {
                const uint64_t lo = pr_xor64((uint64_t)a.w[q], msk);
                const uint64_t hi = pr_xor64((uint64_t)((u128)a.w[q] >> 64), msk);
                a.w[q] += (i128)(((u128)hi << 64) | (u128)lo);
            }
        }
        if (lane < 16) {
            for (int q = 0; q < 6; q++) lds[lane][q] = (u128)(i128)a.s[q];
            for (int q = 0; q < 9; q++) lds[lane][6 + q] = (u128)a.w[q];
        }
        __syncthreads();
        if (lane < PR_NQ) {
            u128 tot = 0;
#pragma unroll
            for (int t = 0; t < 16; t++) tot += lds[t][lane];
            lds[16][lane] = tot;
        }
        __syncthreads();
        if (lane < PR_NQ) {
            if (nch[r] == 1) {
                i128 t[PR_NQ];
                for (int q = 0; q < PR_NQ; q++) t[q] = (i128)lds[16][q];
                props[(int64_t)lane * T.m + r] = pr_output(lane, t, N, qref, F.L);
            } else {
                const u128 v = lds[16][lane];
                unsigned long long* ac = acc + (int64_t)r * PR_ACC;
                if (lane < 6) {
                    atomicAdd(ac + lane, (unsigned long long)(uint64_t)v);
                } else {
                    const unsigned long long lo = (unsigned long long)(uint64_t)v;
                    const unsigned long long hi = (unsigned long long)(uint64_t)(v >> 64);
                    unsigned long long* p = ac + 6 + 2 * (lane - 6);
                    const unsigned long long old = atomicAdd(p, lo);
                    atomicAdd(p + 1, hi + ((old + lo) < old ? 1ull : 0ull));
                }
            }
        }
        __syncthreads();
    }
}

// nodes of more than one chunk: one thread per (node, property)
__global__ void k_pr_final(const float* __restrict__ x, const float* __restrict__ y,
                           const float* __restrict__ z, PrTree T, float L,
                           const int32_t* __restrict__ nch,
                           const unsigned long long* __restrict__ acc,
                           float* __restrict__ props) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= (int64_t)T.m * PR_NQ) return;
    const int32_t r = (int32_t)(g / PR_NQ);
    const int q = (int)(g % PR_NQ);
    if (nch[r] <= 1) return;
    const unsigned long long* ac = acc + (int64_t)r * PR_ACC;
    i128 t[PR_NQ];
    for (int k = 0; k < 6; k++) t[k] = (i128)(int64_t)ac[k];
    for (int k = 0; k < 9; k++)
        t[6 + k] = (i128)(((u128)ac[7 + 2 * k] << 64) | (u128)ac[6 + 2 * k]);
    int32_t qref[3];
    pr_ref(x, y, z, T.minidx[r], qref);
    props[(int64_t)q * T.m + r] = pr_output(q, t, T.size[r], qref, L);
}

__global__ void k_pr_zero_u64(unsigned long long* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

int props_run(const float* x, const float* y, const float* z, const float* vx,
              const float* vy, const float* vz, int64_t n, float L, int64_t m, int64_t nlev,
              const int32_t* level, const int32_t* parent, const int32_t* min_index,
              const int32_t* size, const int32_t* deepest, float* props, hipStream_t st) {
    const int BT = 256;
    PrTree T{level, parent, min_index, size, deepest, (int32_t)m, (int32_t)nlev};
    // chunks: every member of every node is in at most nlev nodes
    const int64_t cap_items = m + (n * nlev) / PR_CH + 1;
    size_t bytes = 0;
    auto add = [&](size_t b) { bytes += arena_round(b); };
    add(24 * (size_t)n);                                  // member records
    add(8 * (size_t)n); add(8 * (size_t)n);               // sort keys in / out
    add(4 * (size_t)n); add(4 * (size_t)n);               // index in / sorted
    add(4 * (size_t)n);                                   // slot of each particle
    for (int k = 0; k < 11; k++) add(4 * ((size_t)m + 1)); // per-node tables
    add(4 * (size_t)cap_items);                           // chunk -> node
    add(4 * ((size_t)nlev + 2));                          // level starts
    add(8 * PR_ACC * (size_t)m);                          // accumulators
    add(scan_temp_bytes(m)); add(sort_temp_bytes(n)); add(256);
    Arena* ar;
    RS_TRY(arena_reserve(AR_BASE, bytes, &ar));
    float2* rec = take<float2>(ar, 3 * (size_t)n);
    uint64_t* kin = take<uint64_t>(ar, n);
    uint64_t* kout = take<uint64_t>(ar, n);
    int32_t* vin = take<int32_t>(ar, n);
    int32_t* perm = take<int32_t>(ar, n);
    int32_t* slot_of = take<int32_t>(ar, n);
    int32_t* childsum = take<int32_t>(ar, m + 1);
    int32_t* cfill = take<int32_t>(ar, m + 1);
    int32_t* own = take<int32_t>(ar, m + 1);
    int32_t* ownscan = take<int32_t>(ar, m + 1);
    int32_t* off = take<int32_t>(ar, m + 1);
    int32_t* nch = take<int32_t>(ar, m + 1);
    int32_t* chunk_off = take<int32_t>(ar, m + 1);
    int32_t* small = take<int32_t>(ar, m + 1);
    int32_t* soff = take<int32_t>(ar, m + 1);
    int32_t* slist = take<int32_t>(ar, m + 1);
    int32_t* lvl0 = take<int32_t>(ar, m + 1);
    int32_t* items = take<int32_t>(ar, cap_items);
    int32_t* lstart = take<int32_t>(ar, nlev + 2);
    unsigned long long* acc = take<unsigned long long>(ar, (size_t)PR_ACC * m);
    void* ctemp = arena_take(ar, scan_temp_bytes(m));
    const size_t stb = sort_temp_bytes(n);
    void* stemp = arena_take(ar, stb);
    // counters: 0 err, 1 level-0 members, 2 chunks, 3 small nodes,
    // 4..5 members of all nodes (64-bit), 6 own total
    int32_t* ctr = take<int32_t>(ar, 16);
    if (!ctr) return RS_EINTERNAL;
    int32_t* hc = nullptr;
    RS_TRY(host_scratch((void**)&hc, 64));

    RS_TRY(fill_i32(ctr, 0, 16, st));
    RS_TRY(fill_i32(lstart, (int32_t)m, nlev + 2, st));
    RS_TRY(fill_i32(childsum, 0, m + 1, st));
    RS_TRY(fill_i32(cfill, 0, m + 1, st));
    const unsigned gm = grid_for(m, BT, 1ll << 31);
    k_pr_check<<<gm, BT, 0, st>>>(T, n, lstart, childsum, ctr);
    unsigned long long* members = reinterpret_cast<unsigned long long*>(ctr + 4);
    k_pr_prep<<<gm, BT, 0, st>>>(T, childsum, nch, small, lvl0, members, ctr);
    RS_HIP(hipGetLastError());
    RS_TRY(scan_exclusive_i32(lvl0, off, m, ctemp, ctr + 1, st));
    RS_TRY(scan_exclusive_i32(nch, chunk_off, m, ctemp, ctr + 2, st));
    RS_TRY(scan_exclusive_i32(small, soff, m, ctemp, ctr + 3, st));
    RS_HIP(hipMemcpyAsync(hc, ctr, 6 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    if (hc[0]) return RS_EINVAL;
    const double member_levels = (double)*reinterpret_cast<unsigned long long*>(hc + 4);
    if ((int64_t)hc[1] > n) return RS_EINVAL;   // level-0 nodes hold more members than particles
    const int32_t total = hc[2], nsmall = hc[3];
    if (total > cap_items) return RS_EINTERNAL;
    for (int64_t l = 1; l < nlev; l++)
        k_pr_offsets<<<1024, BT, 0, st>>>(T, (int32_t)l, lstart, off, cfill);
    k_pr_own<<<gm, BT, 0, st>>>(T, childsum, own);
    RS_HIP(hipGetLastError());
    RS_TRY(scan_exclusive_i32(own, ownscan, m, ctemp, ctr + 6, st));
    const unsigned gn = grid_for(n, BT, 1ll << 31);
    RS_TRY(fill_i32(slot_of, -1, n, st));
    k_pr_keys<<<gn, BT, 0, st>>>(x, y, z, vx, vy, vz, n, L, T, kin, vin, ctr);
    RS_HIP(hipGetLastError());
    int kbits = 1;
    while (kbits < 32 && ((int64_t)1 << kbits) <= m) kbits++;
    RS_TRY(sort_pairs_u64_i32(kin, kout, vin, perm, n, kbits, stemp, stb, st));
    k_pr_slots<<<gn, BT, 0, st>>>(n, T, kout, perm, off, childsum, own, ownscan, slot_of, ctr);
    k_pr_place<<<gn, BT, 0, st>>>(x, y, z, vx, vy, vz, n, T, slot_of, rec);
    k_pr_lists<<<gm, BT, 0, st>>>(T, nch, small, soff, chunk_off, slist, items);
    k_pr_zero_u64<<<grid_for((int64_t)PR_ACC * m, BT, 65536), BT, 0, st>>>(acc,
                                                                         (int64_t)PR_ACC * m);
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemcpyAsync(hc, ctr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    if (hc[0] & 1) return RS_ERANGE;
    if (hc[0]) return RS_EINVAL;

    const int64_t LQ = (int64_t)llrint((double)L * 1048576.0);   // < 2^31 (L < 2048)
    const PrFrame F{(int32_t)(LQ >> 1), (int32_t)LQ, (int32_t)((LQ + 1) >> 1), L};
    prof_begin("halo_props", st);
    if (nsmall > 0)
        k_pr_small<<<grid_for(nsmall, 256, 1ll << 31), 256, 0, st>>>(x, y, z, nsmall, slist, T, F,
                                                                     off, rec, props);
    if (total > 0)
        k_pr_large<<<(unsigned)std::min<int64_t>(total, 1 << 16), 64, 0, st>>>(
            x, y, z, total, items, T, F, off, chunk_off, nch, rec, acc, props);
    k_pr_final<<<grid_for(m * PR_NQ, BT, 1ll << 31), BT, 0, st>>>(x, y, z, T, L, nch, acc,
                                                                 props);
    RS_HIP(hipGetLastError());
    prof_end("halo_props", st, member_levels);
    RS_HIP(hipStreamSynchronize(st));
    return RS_OK;
}

// ---------------------------------------------------------------------------
// seed-halo assignment: seeds are the leaves; a particle whose deepest node
// has children goes to the nearest seed below it under that seed's own
// metric (ties to the smaller node index)
// ---------------------------------------------------------------------------

struct SeedRec {
    float cx, cy, cz, ux, uy, uz, a, c;   // centre, bulk velocity, metric factors
};

// bottom-up: leaf counts of the nodes of level l added to their parents
__global__ void k_sd_leafup(PrTree T, int32_t l, const int32_t* __restrict__ lstart,
                            int32_t* __restrict__ leafcnt) {
    const int32_t b = lstart[l], e = lstart[l + 1];
    for (int32_t r = b + blockIdx.x * blockDim.x + threadIdx.x; r < e;
         r += gridDim.x * blockDim.x)
        atomicAdd(leafcnt + T.parent[r], leafcnt[r]);
}

// top-down: each node's run in the leaf list, carved from its parent's
__global__ void k_sd_leafdown(PrTree T, int32_t l, const int32_t* __restrict__ lstart,
                              const int32_t* __restrict__ leafcnt, int32_t* __restrict__ lfirst,
                              int32_t* __restrict__ lfill) {
    const int32_t b = lstart[l], e = lstart[l + 1];
    for (int32_t r = b + blockIdx.x * blockDim.x + threadIdx.x; r < e;
         r += gridDim.x * blockDim.x) {
        const int32_t p = T.parent[r];
        lfirst[r] = lfirst[p] + atomicAdd(lfill + p, leafcnt[r]);
    }
}

__global__ void k_sd_init(PrTree T, const int32_t* __restrict__ childsum,
                          int32_t* __restrict__ leafcnt, int32_t* __restrict__ err) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= T.m) return;
    if (childsum[r] > T.size[r]) atomicOr(err, 2);
    leafcnt[r] = childsum[r] == 0 ? 1 : 0;
}

__global__ void k_sd_level0(PrTree T, const int32_t* __restrict__ leafcnt,
                            const int32_t* __restrict__ own, const int32_t* __restrict__ childsum,
                            int32_t* __restrict__ l0cnt, int32_t* __restrict__ nitem) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= T.m) return;
    l0cnt[r] = T.level[r] == 0 ? leafcnt[r] : 0;
    nitem[r] = childsum[r] > 0 ? (own[r] + 63) / 64 : 0;
}

__global__ void k_sd_seeds(PrTree T, const int32_t* __restrict__ childsum,
                           const int32_t* __restrict__ lfirst, const float* __restrict__ props,
                           const float* __restrict__ fa, const float* __restrict__ fc,
                           SeedRec* __restrict__ seeds, int32_t* __restrict__ seednode) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= T.m || childsum[r] != 0) return;
    const int32_t q = lfirst[r];
    const int64_t m = T.m;
    seeds[q] = SeedRec{props[r], props[m + r], props[2 * m + r], props[3 * m + r],
                       props[4 * m + r], props[5 * m + r], fa[r], fc[r]};
    seednode[q] = r;
}

__global__ void k_sd_items(PrTree T, const int32_t* __restrict__ nitem,
                           const int32_t* __restrict__ ioff, int32_t* __restrict__ items) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= T.m) return;
    for (int32_t c = 0; c < nitem[r]; c++) items[ioff[r] + c] = r;
}

// particles outside every node (-1) and particles of a seed (the seed)
__global__ void k_sd_direct(int64_t n, PrTree T, const int32_t* __restrict__ childsum,
                            int32_t* __restrict__ halo) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t d = T.deepest[i];
    if (d < 0 || d >= T.m) halo[i] = -1;
    else if (childsum[d] == 0) halo[i] = d;
}

// one wavefront per 64 own particles of a node with children: each lane
// takes one particle, the seeds below the node are read in turn (one
// uniform 32-byte record each) and the nearest is kept
__global__ void __launch_bounds__(64)
k_sd_assign(const float* __restrict__ x, const float* __restrict__ y,
            const float* __restrict__ z, const float* __restrict__ vx,
            const float* __restrict__ vy, const float* __restrict__ vz, int32_t total,
            const int32_t* __restrict__ items, const int32_t* __restrict__ ioff,
            const int32_t* __restrict__ own, const int32_t* __restrict__ ownscan,
            const int32_t* __restrict__ perm, const int32_t* __restrict__ lfirst,
            const int32_t* __restrict__ leafcnt, const SeedRec* __restrict__ seeds,
            const int32_t* __restrict__ seednode, float L, float h,
            int32_t* __restrict__ halo) {
    const int lane = threadIdx.x;
    for (int32_t it = blockIdx.x; it < total; it += gridDim.x) {
        const int32_t r = __builtin_amdgcn_readfirstlane(items[it]);
        const int32_t c = it - ioff[r];
        const int32_t k = c * 64 + lane;
        if (k >= own[r]) continue;
        const int32_t i = perm[ownscan[r] + k];
        const float px = x[i], py = y[i], pz = z[i], pu = vx[i], pv = vy[i], pw = vz[i];
        const int32_t q0 = __builtin_amdgcn_readfirstlane(lfirst[r]);
        const int32_t q1 = q0 + __builtin_amdgcn_readfirstlane(leafcnt[r]);
        float best = INFINITY;
        int32_t bnode = 0x7fffffff;
        for (int32_t q = q0; q < q1; q++) {
            const SeedRec S = seeds[q];
            const int32_t node = seednode[q];
            const float Dx = sum_sq3(min_image(px - S.cx, L, h), min_image(py - S.cy, L, h),
                                     min_image(pz - S.cz, L, h));
            const float Dv = sum_sq3(pu - S.ux, pv - S.uy, pw - S.uz);
            const float d2 = metric(S.a, Dx, S.c, Dv);
            if (d2 < best || (d2 == best && node < bnode)) {
                best = d2;
                bnode = node;
            }
        }
        halo[i] = bnode;
    }
}

int seeds_run(const float* x, const float* y, const float* z, const float* vx,
              const float* vy, const float* vz, int64_t n, float L, int64_t m, int64_t nlev,
              const int32_t* level, const int32_t* parent, const int32_t* min_index,
              const int32_t* size, const int32_t* deepest, const float* fa, const float* fc,
              const float* props, int32_t* halo, hipStream_t st) {
    const int BT = 256;
    PrTree T{level, parent, min_index, size, deepest, (int32_t)m, (int32_t)nlev};
    const int64_t cap_items = m + n / 64 + 1;
    size_t bytes = 0;
    auto add = [&](size_t b) { bytes += arena_round(b); };
    add(8 * (size_t)n); add(8 * (size_t)n);               // sort keys in / out
    add(4 * (size_t)n); add(4 * (size_t)n);               // index in / sorted
    for (int k = 0; k < 10; k++) add(4 * ((size_t)m + 1)); // per-node tables
    add(sizeof(SeedRec) * ((size_t)m + 1));               // seed records
    add(4 * (size_t)cap_items);                           // item -> node
    add(4 * ((size_t)nlev + 2));                          // level starts
    add(scan_temp_bytes(m)); add(sort_temp_bytes(n)); add(256);
    Arena* ar;
    RS_TRY(arena_reserve(AR_BASE, bytes, &ar));
    uint64_t* kin = take<uint64_t>(ar, n);
    uint64_t* kout = take<uint64_t>(ar, n);
    int32_t* vin = take<int32_t>(ar, n);
    int32_t* perm = take<int32_t>(ar, n);
    int32_t* childsum = take<int32_t>(ar, m + 1);
    int32_t* own = take<int32_t>(ar, m + 1);
    int32_t* ownscan = take<int32_t>(ar, m + 1);
    int32_t* leafcnt = take<int32_t>(ar, m + 1);
    int32_t* lfirst = take<int32_t>(ar, m + 1);
    int32_t* lfill = take<int32_t>(ar, m + 1);
    int32_t* l0cnt = take<int32_t>(ar, m + 1);
    int32_t* nitem = take<int32_t>(ar, m + 1);
    int32_t* ioff = take<int32_t>(ar, m + 1);
    int32_t* seednode = take<int32_t>(ar, m + 1);
    SeedRec* seeds = take<SeedRec>(ar, m + 1);
    int32_t* items = take<int32_t>(ar, cap_items);
    int32_t* lstart = take<int32_t>(ar, nlev + 2);
    void* ctemp = arena_take(ar, scan_temp_bytes(m));
    const size_t stb = sort_temp_bytes(n);
    void* stemp = arena_take(ar, stb);
    // counters: 0 err, 1 own total, 2 level-0 leaves, 3 items
    int32_t* ctr = take<int32_t>(ar, 16);
    if (!ctr) return RS_EINTERNAL;
    int32_t* hc = nullptr;
    RS_TRY(host_scratch((void**)&hc, 64));

    RS_TRY(fill_i32(ctr, 0, 16, st));
    RS_TRY(fill_i32(lstart, (int32_t)m, nlev + 2, st));
    RS_TRY(fill_i32(childsum, 0, m + 1, st));
    RS_TRY(fill_i32(lfill, 0, m + 1, st));
    const unsigned gm = grid_for(m, BT, 1ll << 31);
    const unsigned gn = grid_for(n, BT, 1ll << 31);
    k_pr_check<<<gm, BT, 0, st>>>(T, n, lstart, childsum, ctr);
    k_sd_init<<<gm, BT, 0, st>>>(T, childsum, leafcnt, ctr);
    k_pr_own<<<gm, BT, 0, st>>>(T, childsum, own);
    RS_HIP(hipGetLastError());
    RS_TRY(scan_exclusive_i32(own, ownscan, m, ctemp, ctr + 1, st));
    k_pr_keys<<<gn, BT, 0, st>>>(x, y, z, vx, vy, vz, n, L, T, kin, vin, ctr);
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemcpyAsync(hc, ctr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    if (hc[0] & 1) return RS_ERANGE;
    if (hc[0]) return RS_EINVAL;
    int kbits = 1;
    while (kbits < 32 && ((int64_t)1 << kbits) <= m) kbits++;
    RS_TRY(sort_pairs_u64_i32(kin, kout, vin, perm, n, kbits, stemp, stb, st));
    k_pr_slots<<<gn, BT, 0, st>>>(n, T, kout, perm, nullptr, childsum, own, ownscan, nullptr,
                                  ctr);
    for (int64_t l = nlev - 1; l >= 1; l--)
        k_sd_leafup<<<1024, BT, 0, st>>>(T, (int32_t)l, lstart, leafcnt);
    k_sd_level0<<<gm, BT, 0, st>>>(T, leafcnt, own, childsum, l0cnt, nitem);
    RS_HIP(hipGetLastError());
    RS_TRY(scan_exclusive_i32(l0cnt, lfirst, m, ctemp, ctr + 2, st));
    RS_TRY(scan_exclusive_i32(nitem, ioff, m, ctemp, ctr + 3, st));
    for (int64_t l = 1; l < nlev; l++)
        k_sd_leafdown<<<1024, BT, 0, st>>>(T, (int32_t)l, lstart, leafcnt, lfirst, lfill);
    k_sd_seeds<<<gm, BT, 0, st>>>(T, childsum, lfirst, props, fa, fc, seeds, seednode);
    k_sd_items<<<gm, BT, 0, st>>>(T, nitem, ioff, items);
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemcpyAsync(hc, ctr, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    if (hc[0]) return RS_EINVAL;
    const int32_t total = hc[3];
    if (total > cap_items) return RS_EINTERNAL;
    prof_begin("seed_assign", st);
    k_sd_direct<<<gn, BT, 0, st>>>(n, T, childsum, halo);
    if (total > 0)
        k_sd_assign<<<(unsigned)std::min<int64_t>(total, 1 << 16), 64, 0, st>>>(
            x, y, z, vx, vy, vz, total, items, ioff, own, ownscan, perm, lfirst, leafcnt, seeds,
            seednode, L, 0.5f * L, halo);
    RS_HIP(hipGetLastError());
    prof_end("seed_assign", st, (double)n);
    RS_HIP(hipStreamSynchronize(st));
    return RS_OK;
}

}  // namespace rs
