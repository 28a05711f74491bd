// phase.hip -- host orchestration of the hierarchical 6D phase-space FoF
// (subhalo finding inside every 3D FoF halo, paper's Parallelization
// section).
//
//   level 0   groups with >= min_group members become nodes; their members
//             are packed per node (any order -- every result is a pure
//             function of the member set)
//   small     nodes of <= SMALL_MAX members: whole subtree in one workgroup
//             (size-bucketed launches)
//   large     bigger nodes: one level at a time through the tiled pipeline;
//             their small children join the workgroup kernels
//   output    node records are sorted by (level, smallest member index);
//             parents and per-particle deepest nodes are remapped
//
// Forms: RS_BATCHED pushes all groups through each launch; RS_PLAIN walks
// the level-0 groups one at a time (one group per launch sequence).  Both
// run the same kernels and give identical results.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "phase_common.h"

namespace rs {

// ---------------------------------------------------------------------------
// level 0
// ---------------------------------------------------------------------------

// validation + sort keys: (label, index) pairs
__global__ void k_p_keys(const float* __restrict__ x, const float* __restrict__ y,
                         const float* __restrict__ z, const float* __restrict__ vx,
                         const float* __restrict__ vy, const float* __restrict__ vz,
                         const int32_t* __restrict__ lab, int64_t n, float L,
                         uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
                         int32_t* __restrict__ err) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool bad = !(x[i] >= 0.0f && x[i] < L) || !(y[i] >= 0.0f && y[i] < L) ||
               !(z[i] >= 0.0f && z[i] < L);
    bad |= !(fabsf(vx[i]) < 1048576.0f) || !(fabsf(vy[i]) < 1048576.0f) ||
           !(fabsf(vz[i]) < 1048576.0f);
    if (bad) atomicOr(err, 1);
    int32_t l = lab[i];
    if (l < 0 || l >= n) {
        atomicOr(err, 2);
        l = 0;
    }
    keys[i] = (uint64_t)(uint32_t)l;
    vals[i] = (int32_t)i;
}

// run starts of equal labels in the sorted order
__global__ void k_p_runflag(int64_t n, const uint64_t* __restrict__ slab,
                            int32_t* __restrict__ flag) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < n) flag[p] = (p == 0 || slab[p] != slab[p - 1]) ? 1 : 0;
}

__global__ void k_p_runstart(int64_t n, const int32_t* __restrict__ flag,
                             const int32_t* __restrict__ rex, int32_t* __restrict__ rstart) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < n && flag[p]) rstart[rex[p]] = (int32_t)p;
}

__global__ void k_p_keep(int32_t nruns, const int32_t* __restrict__ rstart, int32_t min_group,
                         int32_t* __restrict__ keep, int32_t* __restrict__ klen) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nruns) return;
    int32_t len = rstart[r + 1] - rstart[r];
    bool k = len >= min_group;
    keep[r] = k ? 1 : 0;
    klen[r] = k ? len : 0;
}

// the six phase-space coordinates of every particle interleaved, 24 bytes a
// particle, so that the gather below fetches one record (one or two cache
// lines) per member instead of six scattered values
__global__ void k_p_interleave(int64_t n, const float* __restrict__ x, const float* __restrict__ y,
                               const float* __restrict__ z, const float* __restrict__ vx,
                               const float* __restrict__ vy, const float* __restrict__ vz,
                               float2* __restrict__ rec) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    rec[3 * i] = make_float2(x[i], y[i]);
    rec[3 * i + 1] = make_float2(z[i], vx[i]);
    rec[3 * i + 2] = make_float2(vy[i], vz[i]);
}

// members packed per group in ascending particle index (the sort is stable)
__global__ void k_p_fill(int64_t n, const float2* __restrict__ rec,
                         const int32_t* __restrict__ sidx, const int32_t* __restrict__ flag,
                         const int32_t* __restrict__ rex, const int32_t* __restrict__ rstart,
                         const int32_t* __restrict__ keep, const int32_t* __restrict__ gid,
                         const int32_t* __restrict__ goff, Members A,
                         int32_t* __restrict__ deepest) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t r = rex[p] + flag[p] - 1;
    int32_t i = sidx[p];
    if (!keep[r]) {
        deepest[i] = -1;
        return;
    }
    int64_t pos = (int64_t)goff[r] + (p - rstart[r]);
    const float2 a = rec[3 * (int64_t)i], b = rec[3 * (int64_t)i + 1], c = rec[3 * (int64_t)i + 2];
    A.x[pos] = a.x;
    A.y[pos] = a.y;
    A.z[pos] = b.x;
    A.vx[pos] = b.y;
    A.vy[pos] = c.x;
    A.vz[pos] = c.y;
    A.idx[pos] = i;
    deepest[i] = gid[r];
}

// Percolation of each 3D group: per axis the smallest and largest integer
// displacement of its members from the reference member (the first packed
// member, the smallest index), in the nearest periodic image exactly as for
// the dispersions.  Stored offset by 2^62 so that unsigned atomics order
// them; lanes of one group (members are packed per group) combine first.
constexpr unsigned long long SPAN_OFF = 1ull << 62;

__global__ void k_p_span_init(int32_t G, unsigned long long* __restrict__ span) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < 6 * (int64_t)G) span[i] = (i % 6) < 3 ? ~0ull : 0ull;
}

__global__ void k_p_span(int64_t n, const int32_t* __restrict__ flag,
                         const int32_t* __restrict__ rex, const int32_t* __restrict__ rstart,
                         const int32_t* __restrict__ keep, const int32_t* __restrict__ gid,
                         const int32_t* __restrict__ goff, Members A, int64_t LQ,
                         unsigned long long* __restrict__ span) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool ok = p < n;
    const int32_t r = ok ? rex[p] + flag[p] - 1 : 0;
    ok = ok && keep[r];
    const int32_t g = ok ? gid[r] : -1;
    unsigned long long d[3] = {SPAN_OFF, SPAN_OFF, SPAN_OFF};
    if (ok) {
        const int64_t ref = goff[r], pos = ref + (p - rstart[r]);
        const float* ax3[3] = {A.x, A.y, A.z};
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            int64_t q = quant_pos(ax3[ax][pos]) - quant_pos(ax3[ax][ref]);
            if (2 * q > LQ) q -= LQ;
            else if (2 * q <= -LQ) q += LQ;
            d[ax] = (unsigned long long)(q + (int64_t)SPAN_OFF);
        }
    }
    uint64_t todo = __ballot(ok);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int32_t lg = __shfl(g, leader, 64);
        const bool mine = ok && g == lg;
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            const unsigned long long mn = wave_min_u64(mine ? d[ax] : ~0ull);
            const unsigned long long mx = ~wave_min_u64(mine ? ~d[ax] : ~0ull);
            if ((int)(threadIdx.x & 63) == leader) {
                atomicMin(span + 6 * (int64_t)lg + ax, mn);
                atomicMax(span + 6 * (int64_t)lg + 3 + ax, mx);
            }
        }
        todo &= ~__ballot(mine);
    }
}

// a group percolates when on some axis 2 * (max - min) >= L_Q
__global__ void k_p_wide(int32_t G, const unsigned long long* __restrict__ span, int64_t LQ,
                         int32_t* __restrict__ wide0) {
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    int32_t w = 0;
    for (int ax = 0; ax < 3; ax++) {
        const unsigned long long mn = span[6 * (int64_t)g + ax], mx = span[6 * (int64_t)g + 3 + ax];
        if (2 * (int64_t)(mx - mn) >= LQ) w = 1;
    }
    wide0[g] = w;
}

// level-0 records; small groups into the bucket lists, large ones listed
__global__ void k_p_class(int32_t nruns, const int32_t* __restrict__ rstart,
                          const int32_t* __restrict__ keep, const int32_t* __restrict__ gid,
                          const int32_t* __restrict__ goff, const int32_t* __restrict__ sidx,
                          NodeRec nr, SmallItem* __restrict__ buckets, int64_t stride,
                          int32_t* __restrict__ bcount, ChildOut* __restrict__ large,
                          int32_t* __restrict__ nlarge) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nruns || !keep[r]) return;
    int32_t g = gid[r];
    int32_t sz = rstart[r + 1] - rstart[r];
    int32_t mi = sidx[rstart[r]];
    nr.level[g] = 0;
    nr.minidx[g] = mi;
    nr.parent[g] = -1;
    nr.size[g] = sz;
    if (sz <= SMALL_MAX) {
        int b = sz <= 64 ? 0 : sz <= 256 ? 1 : sz <= 1024 ? 2 : 3;   // small_bucket_of
        int p = atomicAdd(bcount + b, 1);
        buckets[b * stride + p] = SmallItem{g, 0, sz, mi, (int64_t)goff[r]};
    } else {
        int p = atomicAdd(nlarge, 1);
        large[p] = ChildOut{g, sz, mi, 0, (int64_t)goff[r]};
    }
}

// ---------------------------------------------------------------------------
// output assembly
// ---------------------------------------------------------------------------

__global__ void k_o_keys(int32_t m, NodeRec nr, uint64_t* __restrict__ keys,
                         int32_t* __restrict__ vals) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= m) return;
    keys[s] = ((uint64_t)(uint32_t)nr.level[s] << 32) | (uint32_t)nr.minidx[s];
    vals[s] = s;
}

__global__ void k_o_canon(int32_t m, const int32_t* __restrict__ order,
                          int32_t* __restrict__ canon) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < m) canon[order[r]] = r;
}

__global__ void k_o_nodes(int32_t m, const int32_t* __restrict__ order,
                          const int32_t* __restrict__ canon, NodeRec nr, rs_tree t) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    int32_t s = order[r];
    t.level[r] = nr.level[s];
    t.min_index[r] = nr.minidx[s];
    int32_t p = nr.parent[s];
    t.parent[r] = p < 0 ? -1 : canon[p];
    t.size[r] = nr.size[s];
    t.l2[r] = nr.l2[s];
    t.a[r] = nr.a[s];
    t.c[r] = nr.c[s];
    t.sx2[r] = nr.sx2[s];
    t.sv2[r] = nr.sv2[s];
}

// a node carries the percolation flag of its 3D group (level-0 ancestor,
// whose record slot is the group id)
__global__ void k_o_wide(int32_t m, const int32_t* __restrict__ order,
                         const int32_t* __restrict__ tparent, const int32_t* __restrict__ wide0,
                         int32_t* __restrict__ out) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    int32_t a = r;
    while (tparent[a] >= 0) a = tparent[a];
    out[r] = wide0[order[a]];
}

__global__ void k_o_feat(int32_t m, const int32_t* __restrict__ order,
                         const float* __restrict__ feat, float* __restrict__ out) {
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= (int64_t)m * RS_NFEAT) return;
    int32_t r = (int32_t)(q / RS_NFEAT), i = (int32_t)(q % RS_NFEAT);
    out[q] = feat[(int64_t)order[r] * RS_NFEAT + i];
}

__global__ void k_o_deep(int64_t n, const int32_t* __restrict__ deepest,
                         const int32_t* __restrict__ canon, int32_t* __restrict__ out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t d = deepest[i];
    out[i] = d < 0 ? -1 : canon[d];
}

// ---------------------------------------------------------------------------

void tree_release(rs_tree* t) {
    if (!t) return;
    if (t->level) (void)hipFree(t->level);
    free(t);
}

// Side streams (default priority) and ordering events per device, created on
// first use and kept for the process.  Stream 0 takes the level-0 small
// subtrees, stream 1 the small children of each large-node level.
static int side_stream(int which, hipStream_t* s, hipEvent_t* ready, hipEvent_t* done) {
    static hipStream_t g_s[64][2];
    static hipEvent_t g_r[64][2], g_d[64][2];
    int dev = 0;
    RS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64 || which < 0 || which > 1) return RS_EDEVICE;
    if (!g_s[dev][which]) {
        RS_HIP(hipStreamCreateWithFlags(&g_s[dev][which], hipStreamNonBlocking));
        RS_HIP(hipEventCreateWithFlags(&g_r[dev][which], hipEventDisableTiming));
        RS_HIP(hipEventCreateWithFlags(&g_d[dev][which], hipEventDisableTiming));
    }
    *s = g_s[dev][which];
    *ready = g_r[dev][which];
    *done = g_d[dev][which];
    return RS_OK;
}

static int phase_attempt(const float* x, const float* y, const float* z, const float* vx,
                         const float* vy, const float* vz, int64_t n, float L,
                         const int32_t* lab, int32_t min_group, const PhaseParams& pp,
                         uint32_t form, const float* model_host, int64_t cap, rs_tree** out,
                         bool* overflow, hipStream_t st) {
    const int BT = 256;
    *overflow = false;
    // ---- arena 1: level-0 tables, records, output sort ----
    size_t bytes = 0;
    auto add = [&](size_t b) { bytes += arena_round(b); };
    add(24 * (size_t)n);                                       // label keys in, out, index in;
                                                               // then the interleaved records
    add(4 * (size_t)n);                                        // index out
    for (int k = 0; k < 8; k++) add(4 * ((size_t)n + 1));     // flag rex rstart keep klen gid goff deepest
    for (int k = 0; k < 7; k++) add(4 * (size_t)n);           // A
    for (int k = 0; k < 9; k++) add(4 * (size_t)cap);         // records
    add(8 * (size_t)cap); add(8 * (size_t)cap); add(4 * (size_t)cap); add(4 * (size_t)cap);
    add(4 * (size_t)cap);                                      // canon
    const int64_t bstride = n / (min_group > 1 ? min_group : 1) + 2;   // groups per bucket, at most
    add(sizeof(SmallItem) * 4 * (size_t)bstride);              // level-0 buckets
    add(8 * 6 * (size_t)bstride); add(4 * (size_t)bstride);    // group extents, percolation
    add(sizeof(ChildOut) * (size_t)(n / (SMALL_MAX + 1) + 2));
    add(sort_temp_bytes(cap > n ? cap : n)); add(scan_temp_bytes(n)); add(256);
    const bool want_feat = pp.want_feat != 0;
    if (want_feat) add(4 * (size_t)cap * RS_NFEAT);
    const size_t model_floats = 2 * RS_NFEAT + RS_MLP_NPARAM;
    add(4 * model_floats);
    Arena* ar;
    RS_TRY(arena_reserve(AR_BASE, bytes, &ar));
    // the label sort's keys and input indices share one region, which holds
    // the interleaved coordinates once they are consumed
    char* lreg = take<char>(ar, 24 * (size_t)n);
    uint64_t* lkin = reinterpret_cast<uint64_t*>(lreg);
    uint64_t* lkout = reinterpret_cast<uint64_t*>(lreg + 8 * (size_t)n);
    int32_t* lvin = reinterpret_cast<int32_t*>(lreg + 16 * (size_t)n);
    float2* prec = reinterpret_cast<float2*>(lreg);
    int32_t* sidx = take<int32_t>(ar, n);
    int32_t* flag = take<int32_t>(ar, n + 1);
    int32_t* rex = take<int32_t>(ar, n + 1);
    int32_t* rstart = take<int32_t>(ar, n + 1);
    int32_t* keep = take<int32_t>(ar, n + 1);
    int32_t* klen = take<int32_t>(ar, n + 1);
    int32_t* gid = take<int32_t>(ar, n + 1);
    int32_t* goff = take<int32_t>(ar, n + 1);
    int32_t* deepest = take<int32_t>(ar, n + 1);
    Members A;
    A.x = take<float>(ar, n); A.y = take<float>(ar, n); A.z = take<float>(ar, n);
    A.vx = take<float>(ar, n); A.vy = take<float>(ar, n); A.vz = take<float>(ar, n);
    A.idx = take<int32_t>(ar, n);
    NodeRec nr;
    nr.level = take<int32_t>(ar, cap);
    nr.minidx = take<int32_t>(ar, cap);
    nr.parent = take<int32_t>(ar, cap);
    nr.size = take<int32_t>(ar, cap);
    nr.l2 = take<float>(ar, cap);
    nr.a = take<float>(ar, cap);
    nr.c = take<float>(ar, cap);
    nr.sx2 = take<float>(ar, cap);
    nr.sv2 = take<float>(ar, cap);
    nr.cap = (int32_t)cap;
    nr.feat = want_feat ? take<float>(ar, (size_t)cap * RS_NFEAT) : nullptr;
    float* model_dev = take<float>(ar, model_floats);
    uint64_t* okin = take<uint64_t>(ar, cap);
    uint64_t* okout = take<uint64_t>(ar, cap);
    int32_t* ovin = take<int32_t>(ar, cap);
    int32_t* order = take<int32_t>(ar, cap);
    int32_t* canon = take<int32_t>(ar, cap);
    SmallItem* buckets = take<SmallItem>(ar, 4 * bstride);
    unsigned long long* gspan = take<unsigned long long>(ar, 6 * bstride);
    int32_t* wide0 = take<int32_t>(ar, bstride);
    ChildOut* large0 = take<ChildOut>(ar, n / (SMALL_MAX + 1) + 2);
    size_t stb = sort_temp_bytes(cap > n ? cap : n);
    void* stemp = arena_take(ar, stb);
    void* ctemp = arena_take(ar, scan_temp_bytes(n));
    // counters: 0 err, 1 runs, 2 G, 3 node count, 4 overflow, 5 M0, 8..11 buckets, 12 nlarge
    int32_t* ctr = take<int32_t>(ar, 32);
    if (!ctr) return RS_EINTERNAL;
    nr.count = ctr + 3;
    nr.overflow = ctr + 4;
    int32_t* hc = nullptr;
    RS_TRY(host_scratch((void**)&hc, 256));

    unsigned gb = grid_for(n, BT, 1ll << 31);
    RS_HIP(hipMemsetAsync(ctr, 0, 32 * sizeof(int32_t), st));
    k_p_keys<<<gb, BT, 0, st>>>(x, y, z, vx, vy, vz, lab, n, L, lkin, lvin, ctr);
    RS_HIP(hipGetLastError());
    int lbits = 1;
    while (lbits < 31 && ((int64_t)1 << lbits) < n) lbits++;
    RS_TRY(sort_pairs_u64_i32(lkin, lkout, lvin, sidx, n, lbits, stemp, stb, st));
    k_p_runflag<<<gb, BT, 0, st>>>(n, lkout, flag);
    k_p_interleave<<<gb, BT, 0, st>>>(n, x, y, z, vx, vy, vz, prec);
    RS_HIP(hipGetLastError());
    RS_TRY(scan_exclusive_i32(flag, rex, n, ctemp, ctr + 1, st));
    k_p_runstart<<<gb, BT, 0, st>>>(n, flag, rex, rstart);
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemcpyAsync(hc, ctr, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    if (hc[0] & 2) return RS_EINVAL;
    if (hc[0] & 1) return RS_ERANGE;
    const int32_t nruns = hc[1];
    RS_TRY(fill_i32(rstart + nruns, (int32_t)n, 1, st));
    k_p_keep<<<grid_for(nruns, BT, 1ll << 31), BT, 0, st>>>(nruns, rstart, min_group, keep, klen);
    RS_HIP(hipGetLastError());
    RS_TRY(scan_exclusive_i32(keep, gid, nruns, ctemp, ctr + 2, st));
    RS_TRY(scan_exclusive_i32(klen, goff, nruns, ctemp, ctr + 5, st));
    RS_HIP(hipMemcpyAsync(hc, ctr, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    const int32_t G = hc[2];
    if (G > cap) {
        *overflow = true;
        return RS_OK;
    }
    k_p_fill<<<gb, BT, 0, st>>>(n, prec, sidx, flag, rex, rstart, keep, gid, goff, A, deepest);
    k_p_class<<<grid_for(nruns, BT, 1ll << 31), BT, 0, st>>>(nruns, rstart, keep, gid, goff, sidx,
                                                              nr, buckets, bstride, ctr + 8,
                                                              large0, ctr + 12);
    RS_HIP(hipGetLastError());
    // percolation flags of the groups; only the output reads them, so the
    // batched form runs them on the side stream of the level-0 subtrees
    auto span_pass = [&](hipStream_t s) {
        if (G <= 0) return;
        k_p_span_init<<<grid_for(6 * (int64_t)G, BT, 1ll << 31), BT, 0, s>>>(G, gspan);
        k_p_span<<<gb, BT, 0, s>>>(n, flag, rex, rstart, keep, gid, goff, A, pp.LQ, gspan);
        k_p_wide<<<grid_for(G, BT, 1ll << 31), BT, 0, s>>>(G, gspan, pp.LQ, wide0);
    };
    RS_TRY(fill_i32(nr.count, G, 1, st));
    RS_HIP(hipMemcpyAsync(hc, ctr, 16 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    const int32_t nlarge = hc[12];
    int32_t bcnt[4] = {hc[8], hc[9], hc[10], hc[11]};
    std::vector<ChildOut> large(nlarge);
    if (nlarge > 0) {
        RS_HIP(hipMemcpyAsync(large.data(), large0, sizeof(ChildOut) * nlarge,
                              hipMemcpyDeviceToHost, st));
        RS_HIP(hipStreamSynchronize(st));
        std::sort(large.begin(), large.end(),
                  [](const ChildOut& a, const ChildOut& b) { return a.slot < b.slot; });
    }
    int64_t mlarge = 0, mmax = 0;
    for (auto& c : large) {
        mlarge += c.size;
        mmax = c.size > mmax ? c.size : mmax;
    }

    // ---- large-node work space (arena 2) ----
    // Members one pass of the level pipeline holds: every large group at once
    // when the device has room, else consecutive chunks of groups (each group
    // whole), sized from the memory this call can obtain.  The plain form
    // walks one group at a time and needs room for the largest only.
    int64_t mcap = form == RS_PLAIN ? mmax : mlarge;
    if (mcap > mmax) {
        size_t budget = 0;
        RS_TRY(device_budget((1u << AR_LARGE) | (1u << AR_TREE), &budget));
        const int64_t probe = (int64_t)1 << 24;
        const double per = (double)large_work_bytes(probe, pp.min_sub) / (double)probe + 16.0;
        const size_t keep = (size_t)cap * (9 * 4 + 4 * (want_feat ? RS_NFEAT : 0)) +
                            (size_t)n * 4 + ((size_t)2 << 30);
        const int64_t fit = budget > keep ? (int64_t)((double)(budget - keep) / per) : 0;
        if (fit < mcap) mcap = fit > mmax ? fit : mmax;
        // test hook: a smaller chunk budget exercises the chunked path on small inputs
        if (const char* e = getenv("RS_DEBUG_CHUNK_MEMBERS")) {
            const int64_t v = atoll(e);
            if (v > 0 && v < mcap) mcap = v > mmax ? v : mmax;
        }
    }
    LargeWork lw;
    int64_t n_acc = 0, n_fb = 0;
    if (nlarge > 0) {
        Arena* ar2;
        RS_TRY(arena_reserve(AR_LARGE, large_work_bytes(mcap, pp.min_sub), &ar2));
        RS_TRY(large_work_carve(ar2, mcap, pp.min_sub, &lw));
        if (form == RS_LEARNED) {
            RS_HIP(hipMemcpyAsync(model_dev, model_host, 4 * model_floats, hipMemcpyHostToDevice,
                                  st));
            lw.model = model_dev;
        }
    }

    if (form == RS_PLAIN) {
        // one level-0 group per launch sequence, in slot order
        std::vector<SmallItem> hs;
        for (int b = 0; b < 4; b++) {
            size_t o = hs.size();
            hs.resize(o + bcnt[b]);
            if (bcnt[b] > 0)
                RS_HIP(hipMemcpyAsync(hs.data() + o, buckets + b * bstride,
                                      sizeof(SmallItem) * bcnt[b], hipMemcpyDeviceToHost, st));
        }
        RS_HIP(hipStreamSynchronize(st));
        std::sort(hs.begin(), hs.end(),
                  [](const SmallItem& a, const SmallItem& b) { return a.slot < b.slot; });
        span_pass(st);
        RS_HIP(hipGetLastError());
        SmallItem* one = buckets;   // reuse: the host copy is complete
        size_t si = 0, li = 0;
        while (si < hs.size() || li < large.size()) {
            bool take_small =
                li >= large.size() || (si < hs.size() && hs[si].slot < large[li].slot);
            if (take_small) {
                RS_HIP(hipMemcpyAsync(one, &hs[si], sizeof(SmallItem), hipMemcpyHostToDevice, st));
                RS_TRY(run_small_bucket(small_bucket_of(hs[si].size), one, 1, A, nr, pp, deepest,
                                        st));
                RS_HIP(hipStreamSynchronize(st));
                si++;
            } else {
                std::vector<ChildOut> cur{large[li]}, nxt;
                const Members* in = &A;
                while (!cur.empty()) {
                    RS_TRY(large_level(&lw, cur, *in, x, y, z, pp, nr, deepest, &nxt, &n_acc,
                                       &n_fb, st));
                    cur.swap(nxt);
                    in = &lw.SN;
                }
                li++;
            }
        }
    } else {
        // The level-0 subtrees of the small groups run on a side stream while
        // the large-node levels run on the caller's: they read the level-0
        // members only, write disjoint particles' deepest nodes and take node
        // record slots atomically, so the two overlap freely and the result
        // does not depend on their interleaving.  The percolation pass follows
        // them there, away from the start of the first large-node level.
        hipStream_t s2 = nullptr;
        hipEvent_t ready = nullptr, done = nullptr;
        RS_TRY(side_stream(0, &s2, &ready, &done));
        RS_TRY(side_stream(1, &lw.side, &lw.side_ready, &lw.side_done));
        lw.side_pending = false;
        RS_HIP(hipEventRecord(ready, st));
        RS_HIP(hipStreamWaitEvent(s2, ready, 0));
        int rc = RS_OK;
        for (int b = 3; b >= 0 && rc == RS_OK; b--)
            rc = run_small_bucket(b, buckets + b * bstride, bcnt[b], A, nr, pp, deepest, s2,
                                  "phase_small_level0");
        span_pass(s2);
        if (rc == RS_OK && hipGetLastError() != hipSuccess) rc = RS_EDEVICE;
        size_t li = 0;
        while (rc == RS_OK && li < large.size()) {
            std::vector<ChildOut> cur, nxt;
            int64_t sum = 0;
            while (li < large.size() && (cur.empty() || sum + large[li].size <= mcap)) {
                sum += large[li].size;
                cur.push_back(large[li++]);
            }
            const Members* in = &A;
            while (rc == RS_OK && !cur.empty()) {
                rc = large_level(&lw, cur, *in, x, y, z, pp, nr, deepest, &nxt, &n_acc, &n_fb,
                                 st);
                cur.swap(nxt);
                in = &lw.SN;
            }
        }
        // join (also on failure, so nothing runs on after the call returns)
        if (hipEventRecord(done, s2) != hipSuccess ||
            hipStreamWaitEvent(st, done, 0) != hipSuccess ||
            (lw.side_pending && hipStreamWaitEvent(st, lw.side_done, 0) != hipSuccess)) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(s2);
            (void)hipStreamSynchronize(lw.side);
            return rc != RS_OK ? rc : RS_EDEVICE;
        }
        if (rc != RS_OK) {
            (void)hipStreamSynchronize(s2);
            (void)hipStreamSynchronize(lw.side);
            return rc;
        }
    }

    // ---- output ----
    RS_HIP(hipMemcpyAsync(hc, ctr + 3, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    if (hc[1]) {
        *overflow = true;
        return RS_OK;
    }
    const int32_t m = hc[0];
    if (m > 0) {
        k_o_keys<<<grid_for(m, BT, 1ll << 31), BT, 0, st>>>(m, nr, okin, ovin);
        RS_HIP(hipGetLastError());
        RS_TRY(sort_pairs_u64_i32(okin, okout, ovin, order, m, 48, stemp, stb,
                                  st));
        k_o_canon<<<grid_for(m, BT, 1ll << 31), BT, 0, st>>>(m, order, canon);
        RS_HIP(hipGetLastError());
    }
    size_t nodes_bytes = arena_round(4 * (size_t)(m > 0 ? m : 1));
    size_t feat_bytes = want_feat ? arena_round(4 * (size_t)(m > 0 ? m : 1) * RS_NFEAT) : 0;
    size_t total = 10 * nodes_bytes + arena_round(4 * (size_t)(n > 0 ? n : 1)) + feat_bytes;
    rs_tree* t = (rs_tree*)calloc(1, sizeof(rs_tree));
    if (!t) return RS_ENOMEM;
    char* blk = nullptr;
    hipError_t e = hipMalloc((void**)&blk, total);
    if (e != hipSuccess) {
        // the level work spaces are done with; give them back and try again
        (void)hipGetLastError();
        if (arena_release(AR_LARGE) != RS_OK || arena_release(AR_TREE) != RS_OK ||
            hipMalloc((void**)&blk, total) != hipSuccess) {
            (void)hipGetLastError();
            free(t);
            return RS_ENOMEM;
        }
    }
    t->n_nodes = m;
    t->n_particles = n;
    t->level = (int32_t*)(blk + 0 * nodes_bytes);
    t->min_index = (int32_t*)(blk + 1 * nodes_bytes);
    t->parent = (int32_t*)(blk + 2 * nodes_bytes);
    t->size = (int32_t*)(blk + 3 * nodes_bytes);
    t->l2 = (float*)(blk + 4 * nodes_bytes);
    t->a = (float*)(blk + 5 * nodes_bytes);
    t->c = (float*)(blk + 6 * nodes_bytes);
    t->sx2 = (float*)(blk + 7 * nodes_bytes);
    t->sv2 = (float*)(blk + 8 * nodes_bytes);
    t->wide = (int32_t*)(blk + 9 * nodes_bytes);
    t->deepest = (int32_t*)(blk + 10 * nodes_bytes);
    t->features = want_feat
        ? (float*)(blk + 10 * nodes_bytes + arena_round(4 * (size_t)(n > 0 ? n : 1)))
        : nullptr;
    t->n_accepted = n_acc;
    t->n_fallback = n_fb;
    int rc = RS_OK;
    if (want_feat && m > 0)
        k_o_feat<<<grid_for((int64_t)m * RS_NFEAT, BT, 1ll << 31), BT, 0, st>>>(m, order, nr.feat,
                                                                             t->features);
    if (m > 0) {
        k_o_nodes<<<grid_for(m, BT, 1ll << 31), BT, 0, st>>>(m, order, canon, nr, *t);
        k_o_wide<<<grid_for(m, BT, 1ll << 31), BT, 0, st>>>(m, order, t->parent, wide0, t->wide);
    }
    if (n > 0) k_o_deep<<<gb, BT, 0, st>>>(n, deepest, canon, t->deepest);
    if (hipGetLastError() != hipSuccess) rc = RS_EDEVICE;
    int32_t last_level = -1;
    if (rc == RS_OK && m > 0) {
        if (hipMemcpyAsync(&last_level, t->level + (m - 1), sizeof(int32_t),
                           hipMemcpyDeviceToHost, st) != hipSuccess)
            rc = RS_EDEVICE;
    }
    if (rc == RS_OK && hipStreamSynchronize(st) != hipSuccess) rc = RS_EDEVICE;
    if (rc != RS_OK) {
        tree_release(t);
        return rc;
    }
    t->n_levels = last_level + 1;
    *out = t;
    return RS_OK;
}

int phase_run(const float* x, const float* y, const float* z, const float* vx,
              const float* vy, const float* vz, int64_t n, float L, const int32_t* labels,
              int32_t min_group, int32_t min_sub, double f, uint32_t flags, const void* model,
              rs_tree** out, hipStream_t st) {
    const uint32_t form = flags & 0xffu;
    const float* model_host = nullptr;
    if (form == RS_LEARNED) {
        if (!model || memcmp(model, "RSM1", 4) != 0) return RS_EINVAL;
        model_host = reinterpret_cast<const float*>(static_cast<const char*>(model) + 4);
    }
    PhaseParams pp;
    pp.want_feat = (flags & RS_FEATURES) ? 1 : 0;
    pp.L = L;
    pp.h = 0.5f * L;
    pp.LQ = (int64_t)rint((double)L * 1048576.0);
    pp.min_sub = min_sub;
    pp.f_ppm = llround(f * 1e6);
    int64_t cap = n / (min_group > 1 ? min_group : 1) + 4 * (n / (min_sub > 1 ? min_sub : 1)) / 3 +
                  1024;
    if (cap > 0x7ffffff0ll) cap = 0x7ffffff0ll;
    for (int attempt = 0; attempt < 8; attempt++) {
        bool overflow = false;
        rs_tree* t = nullptr;
        RS_TRY(phase_attempt(x, y, z, vx, vy, vz, n, L, labels, min_group, pp, form, model_host,
                             cap, &t, &overflow, st));
        if (!overflow) {
            *out = t;
            return RS_OK;
        }
        if (cap >= 0x7ffffff0ll) return RS_EINTERNAL;
        cap = cap * 2 > 0x7ffffff0ll ? 0x7ffffff0ll : cap * 2;
    }
    return RS_EINTERNAL;
}

}  // namespace rs
